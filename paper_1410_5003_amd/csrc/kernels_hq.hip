// Blocked Householder least squares for the per-layer Schur eliminations
// (Sec. 3.2: the products Q^+ C are obtained from a backward-stable dense
// least-squares solve, never from an explicit pseudo-inverse).  The problem
// solved is the Tikhonov-stacked one, min ||Q X - C||^2 + mu^2 ||X||^2,
// i.e. the QR factorisation of [Q; mu I] applied to [C; 0].
//
//   hq_prep_kernel     mu = mu_rel ||Q||_F and the mu I rows;
//   hq_panel_kernel    Householder QR of a 16-column panel in LDS (one
//                      wavefront per column), and the triangular factor T of
//                      its block reflector H = I - V T V^H (compact WY form);
//                      extra workgroups of the launch assemble independent
//                      tiles on the compute units the panels leave idle;
//   hq_update_kernel   the later columns of S: Y <- H^H Y = Y - V T^H (V^H Y),
//                      16 columns per workgroup of 8 wavefronts, the tile in
//                      registers in the matrix-core accumulator layout;
//   hq_rhs_kernel      after the last panel, one workgroup per 16 right-hand
//                      sides: the (M x 16) tile stays in registers while
//                      every block reflector is applied to it, and
//                      R X = (Q^H C)[0:c] is solved by 16-row blocks in LDS
//                      (substitution inside each diagonal block, products
//                      on the FP64 matrix cores elsewhere).  The right-hand
//                      sides cross HBM once instead of once per panel.
#include <algorithm>

#include "internal.hpp"

namespace mlh {

__device__ inline double2 hld(const cplx* p) { return ldc(p); }
__device__ inline void hst(cplx* p, double2 v) { stc(p, v.x, v.y); }

__device__ inline double hwave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void hq_prep_kernel(const HqDesc* __restrict__ descs) {
  const HqDesc& D = descs[blockIdx.x];
  const int m = D.m, c = D.c, M = m + c;
  __shared__ double red[4];
  double acc = 0.0;
#pragma unroll 8
  for (int e = threadIdx.x; e < m * c; e += 256) {
    const double2 x = hld(D.A + (size_t)(e / m) * M + (e % m));
    acc += x.x * x.x + x.y * x.y;
  }
  acc = hwave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  const double mu = D.mu_rel * sqrt(red[0] + red[1] + red[2] + red[3]);
  for (int e = threadIdx.x; e < c * c; e += 256) {
    const int r = e % c, col = e / c;
    hst(D.A + (size_t)col * M + m + r, make_double2(r == col ? mu : 0.0, 0.0));
  }
}

// sum of v over the 16 lanes of each DPP row (lanes 16 m .. 16 m + 15); the
// total lands in the row's last lane
template <int CTRL>
__device__ inline double dpp_shr_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffff), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)((unsigned long long)b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ inline double row16_sum(double v) {
  v += dpp_shr_d<0x111>(v);  // row_shr:1
  v += dpp_shr_d<0x112>(v);  // row_shr:2
  v += dpp_shr_d<0x114>(v);  // row_shr:4
  v += dpp_shr_d<0x118>(v);  // row_shr:8
  return v;
}
template <int CTRL, int ROWS>
__device__ inline double dpp_rows_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffff), CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)((unsigned long long)b >> 32), CTRL, ROWS, 0xf, true);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
// lane R's value within each row of 16 lanes (DPP row_newbcast)
__device__ inline double row_bcast16(double v, int R) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(unsigned)(b & 0xffffffff), hi = (int)(unsigned)((unsigned long long)b >> 32);
#define MLH_BCAST16(n)                                             \
  case n:                                                          \
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x150 + n, 0xf, 0xf, false); \
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x150 + n, 0xf, 0xf, false); \
    break;
  switch (R) {
    MLH_BCAST16(0) MLH_BCAST16(1) MLH_BCAST16(2) MLH_BCAST16(3) MLH_BCAST16(4) MLH_BCAST16(5) MLH_BCAST16(6)
    MLH_BCAST16(7) MLH_BCAST16(8) MLH_BCAST16(9) MLH_BCAST16(10) MLH_BCAST16(11) MLH_BCAST16(12) MLH_BCAST16(13)
    MLH_BCAST16(14) MLH_BCAST16(15)
  }
#undef MLH_BCAST16
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

// sum of v over the wavefront, returned in every lane (wave-uniform)
__device__ inline double wave64_sum(double v) {
  v = row16_sum(v);                   // lane 15 of each row: the row's sum
  v += dpp_rows_d<0x142, 0xa>(v);     // row_bcast:15 into rows 1, 3
  v += dpp_rows_d<0x143, 0xc>(v);     // row_bcast:31 into rows 2, 3 -> lane 63: the total
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffff), 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | lo);
}

// Panel rows k..M-1 of columns k..k+15 in LDS (stride 17 against bank
// conflicts).  Wave j owns column j and lane q the rows congruent to q modulo
// 64 below the current reflector, so each column step is one pass (the norm
// of column i and the raw products of column i with the later columns),
// wavefront sums by DPP, one barrier, and one update pass.  The scaling of
// column i into its Householder vector is deferred to the next pass, which
// does not read that column.
constexpr int kHqPanelThreads = 64 * kHqNb;
// Workgroups from n on assemble tiles [asm_t0, asm_t1) of an independent
// job list, four per workgroup, on the compute units the n panels leave
// idle.
__global__ __launch_bounds__(kHqPanelThreads) void hq_panel_kernel(const HqDesc* __restrict__ descs, int n, int k,
                                                                   const AsmJob* __restrict__ asm_jobs,
                                                                   int asm_njobs, int asm_t0, int asm_t1) {
  if ((int)blockIdx.x >= n) {
    const int t = asm_t0 + ((int)blockIdx.x - n) * (kHqPanelThreads / 256) + (int)(threadIdx.x >> 8);
    if (t < asm_t1) assemble_one<kAsmTile / 512>(asm_jobs, asm_njobs, t, (int)(threadIdx.x & 255));
    return;
  }
  const HqDesc& D = descs[blockIdx.x];
  const int c = D.c, M = D.m + c;
  if (k >= c) return;
  const int nb = min(kHqNb, c - k);
  const int L = M - k;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int jc = wave;  // the column this wave owns
  __shared__ double2 pan[kHqMaxRows][kHqNb + 1];
  __shared__ double2 red[2][kHqNb];
  __shared__ double2 tau[kHqNb], scl[kHqNb];
  __shared__ double2 gram[kHqNb][kHqNb + 1];
  __shared__ double2 T[kHqNb][kHqNb + 1];
  cplx* A = D.A;
  // eight loads in flight per thread (clamped addresses, no guarding branch)
  for (int e0 = tid; e0 < L * kHqNb; e0 += kHqPanelThreads * 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + kHqPanelThreads * u, L * kHqNb - 1);
      v[u] = hld(A + (uint32_t)((k + min(e / L, nb - 1)) * M + k + e % L));
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + kHqPanelThreads * u;
      if (e < L * kHqNb) pan[e % L][e / L] = e / L < nb ? v[u] : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    const int buf = i & 1;
    // deferred: column i - 1 becomes its Householder vector
    if (i > 0 && jc == i - 1) {
      const double2 sc = scl[i - 1];
      for (int r = i + lane; r < L; r += 64) {
        const double2 x = pan[r][i - 1];
        pan[r][i - 1] = make_double2(x.x * sc.x - x.y * sc.y, x.x * sc.y + x.y * sc.x);
      }
    }
    // pass 1: |x|^2 below the diagonal of column i; raw products of column i
    // with the later columns (rows below i)
    if (jc >= i) {
      double ar = 0.0, ai = 0.0;
      for (int r = i + 1 + lane; r < L; r += 64) {
        const double2 x = pan[r][i];
        if (jc == i) {
          ar += x.x * x.x + x.y * x.y;
        } else {
          const double2 y = pan[r][jc];
          ar += x.x * y.x + x.y * y.y;  // conj(x) y
          ai += x.x * y.y - x.y * y.x;
        }
      }
      ar = wave64_sum(ar);
      ai = wave64_sum(ai);
      if (lane == 0) red[buf][jc] = make_double2(ar, ai);
    }
    __syncthreads();
    // the reflector of column i, formed identically in every thread
    const double xn2 = red[buf][i].x;
    const double2 al = pan[i][i];
    double tr = 0.0, ti = 0.0, sr = 1.0, si = 0.0, beta = al.x;
    if (!(xn2 == 0.0 && al.y == 0.0)) {
      beta = -copysign(sqrt(al.x * al.x + al.y * al.y + xn2), al.x);
      tr = (beta - al.x) / beta;
      ti = -al.y / beta;
      const double dr = al.x - beta, di = al.y;
      const double den = dr * dr + di * di;
      sr = dr / den;
      si = -di / den;
    }
    // pass 2: H_i^H on the later columns: w = y_i + conj(s) raw, u = conj(tau) w,
    // y_i -= u, y_r -= s x_r u
    if (jc > i && jc < kHqNb) {
      const double2 raw = red[buf][jc], yi = pan[i][jc];
      const double wr = yi.x + sr * raw.x + si * raw.y, wi = yi.y + sr * raw.y - si * raw.x;
      const double ur = tr * wr + ti * wi, ui = tr * wi - ti * wr;
      const double vr = sr * ur - si * ui, vi = sr * ui + si * ur;  // s u
      if (lane == 0) pan[i][jc] = make_double2(yi.x - ur, yi.y - ui);
      for (int r = i + 1 + lane; r < L; r += 64) {
        const double2 x = pan[r][i];
        double2 y = pan[r][jc];
        y.x -= x.x * vr - x.y * vi;
        y.y -= x.x * vi + x.y * vr;
        pan[r][jc] = y;
      }
    }
    if (tid == 0) {
      tau[i] = make_double2(tr, ti);
      scl[i] = make_double2(sr, si);
    }
    __syncthreads();
    if (tid == 0) pan[i][i] = make_double2(beta, 0.0);  // column i is not read again until scaled
  }
  if (jc == nb - 1) {  // the last column's scaling
    const double2 sc = scl[nb - 1];
    for (int r = nb + lane; r < L; r += 64) {
      const double2 x = pan[r][nb - 1];
      pan[r][nb - 1] = make_double2(x.x * sc.x - x.y * sc.y, x.x * sc.y + x.y * sc.x);
    }
  }
  __syncthreads();
  // Gram matrix G = V^H V (V unit lower trapezoidal): wave b sums
  // conj(v_a) v_b over its lanes' rows for every a < b
  if (jc < nb) {
    double2 g[kHqNb];
#pragma unroll
    for (int a = 0; a < kHqNb; ++a) g[a] = make_double2(0.0, 0.0);
    for (int r = jc + lane; r < L; r += 64) {
      const double2 vb = r == jc ? make_double2(1.0, 0.0) : pan[r][jc];
#pragma unroll
      for (int a = 0; a < kHqNb; ++a) {
        if (a < jc) {
          const double2 va = r == a ? make_double2(1.0, 0.0) : pan[r][a];  // r >= jc > a
          g[a].x += va.x * vb.x + va.y * vb.y;
          g[a].y += va.x * vb.y - va.y * vb.x;
        }
      }
    }
#pragma unroll
    for (int a = 0; a < kHqNb; ++a) {
      if (a < jc) {  // wave-uniform
        const double gr = wave64_sum(g[a].x), gi = wave64_sum(g[a].y);
        if (lane == 0) gram[a][jc] = make_double2(gr, gi);
      }
    }
  }
  __syncthreads();
  // T: T[i][i] = tau_i ; T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]  (wave 0,
  // lane a computes row a)
  if (wave == 0) {
    for (int e = lane; e < kHqNb * kHqNb; e += 64) T[e % kHqNb][e / kHqNb] = make_double2(0.0, 0.0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int i = 0; i < nb; ++i) {
      const double2 ti = tau[i];
      if (lane < i) {
        double2 sacc = make_double2(0.0, 0.0);
        for (int q = lane; q < i; ++q) {
          const double2 x = T[lane][q], gg = gram[q][i];
          sacc.x += x.x * gg.x - x.y * gg.y;
          sacc.y += x.x * gg.y + x.y * gg.x;
        }
        T[lane][i] = make_double2(-(ti.x * sacc.x - ti.y * sacc.y), -(ti.x * sacc.y + ti.y * sacc.x));
      }
      if (lane == i) T[i][i] = ti;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  const int pidx = k / kHqNb;
  for (int e = tid; e < kHqNb * kHqNb; e += kHqPanelThreads)
    hst(D.T + (size_t)pidx * kHqNb * kHqNb + e, T[e % kHqNb][e / kHqNb]);
  for (int e = tid; e < L * nb; e += kHqPanelThreads) {
    const int r = e % L, j = e / L;
    hst(A + (size_t)(k + j) * M + k + r, pan[r][j]);
  }
}

typedef double hvec4 __attribute__((ext_vector_type(4)));

// V of panel k as an MFMA operand value, column i, row r (global): unit
// diagonal, zeros above it and past row M, Householder vectors below.  In
// two parts, so that a load can be in flight while other work runs:
// hq_v_raw loads the stored entry at clamped indices (inside the panel's
// columns and the M rows), hq_v_mask turns it into V's value.
__device__ inline double2 hq_v_raw(const cplx* A, int M, int k, int nb, int r, int i) {
  return hld(A + (size_t)(k + min(i, nb - 1)) * M + min(r, M - 1));
}
__device__ inline double2 hq_v_mask(double2 raw, int M, int k, int nb, int r, int i) {
  if (i >= nb || r < k + i || r >= M) return make_double2(0.0, 0.0);
  if (r == k + i) return make_double2(1.0, 0.0);
  return raw;
}

constexpr int kHqRhsCols = 16;
constexpr int kHqRhsWaves = 8;
static_assert(kHqRhsSmallRows == kHqRhsWaves * 3 * 16 && kHqMaxRows <= kHqRhsWaves * 4 * 16, "row blocks per wave");

// complex 16 x 16 x 4 step of D += op(A) B with three real MFMA products
// (T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi); D = (T1 - T2, T3 - T1 - T2)):
// callers pass Ai = -Im(A) for conj(A)
struct Cacc {
  hvec4 t1, t2, t3;
};
__device__ inline void cacc_zero(Cacc& c) {
  c.t1 = hvec4{0, 0, 0, 0};
  c.t2 = hvec4{0, 0, 0, 0};
  c.t3 = hvec4{0, 0, 0, 0};
}
__device__ inline void cacc_step(Cacc& c, double ar, double ai, double br, double bi) {
  c.t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, c.t1, 0, 0, 0);
  c.t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, c.t2, 0, 0, 0);
  c.t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, br + bi, c.t3, 0, 0, 0);
}

// One block reflector H = I - V T V^H of panel k applied to the M x 16 tile
// (yr, yi) that the eight waves of the workgroup hold in registers:
// Y <- H^H Y = Y - V T^H (V^H Y).  Every wave of the workgroup calls it.
template <int kHqRhsRbw>
__device__ __forceinline__ void hq_apply_panel(hvec4 (&yr)[kHqRhsRbw], hvec4 (&yi)[kHqRhsRbw], const cplx* A, int M,
                                               int k, int nb, const cplx* Tp, double* red) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  // V operands of this wave's row blocks: vh for V^H (lane: reflector lr,
  // row 4 kk + lq), all loaded at once; vv for V (lane: row lr, reflector
  // 4 kk + lq) in step 3, one row block ahead of the products, so that the
  // two layouts are never held together (holding both spilled the tile Y
  // inside the panel loop).  Loads are raw; each block's values are masked
  // just before its products (scheduling barriers keep the selects there),
  // so the wave waits for one block's loads at a time.
  double2 vh[kHqRhsRbw][4];
#pragma unroll
  for (int j = 0; j < kHqRhsRbw; ++j) {
    const int r0 = (wave + kHqRhsWaves * j) * 16;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) vh[j][kk] = hq_v_raw(A, M, k, nb, r0 + 4 * kk + lq, lr);
  }
  // 1. partial w = V^H Y over this wave's rows
  Cacc w;
  cacc_zero(w);
#pragma unroll
  for (int j = 0; j < kHqRhsRbw; ++j) {
    const int r0 = (wave + kHqRhsWaves * j) * 16;
    __builtin_amdgcn_sched_barrier(0);
    if (r0 >= M) break;
    if (r0 + 15 < k) continue;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double2 v = hq_v_mask(vh[j][kk], M, k, nb, r0 + 4 * kk + lq, lr);
      cacc_step(w, v.x, -v.y, yr[j][kk], yi[j][kk]);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  // T of the panel (lane: T[4 kk + lq][lr]), in flight across the reduction
  double2 tt[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) tt[kk] = hld(Tp + (size_t)lr * kHqNb + 4 * kk + lq);
  // red: this panel's buffer of partial sums
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    red[((wave * 2 + 0) * 4 + q) * 64 + lane] = w.t1[q] - w.t2[q];
    red[((wave * 2 + 1) * 4 + q) * 64 + lane] = w.t3[q] - w.t1[q] - w.t2[q];
  }
  __syncthreads();
  // 2. full w (register q: reflector 4 q + lq, column lr), u = T^H w
  double wr[4], wi[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int v = 0; v < kHqRhsWaves; ++v) {
      a += red[((v * 2 + 0) * 4 + q) * 64 + lane];
      b += red[((v * 2 + 1) * 4 + q) * 64 + lane];
    }
    wr[q] = a;
    wi[q] = b;
  }
  // the first row block's V for step 3, in flight during u = T^H w
  double2 vv[2][4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) vv[0][kk] = hq_v_raw(A, M, k, nb, wave * 16 + lr, 4 * kk + lq);
  Cacc u;
  cacc_zero(u);
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) cacc_step(u, tt[kk].x, -tt[kk].y, wr[kk], wi[kk]);  // A = conj(T)^T
  double ur[4], ui[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ur[q] = u.t1[q] - u.t2[q];
    ui[q] = u.t3[q] - u.t1[q] - u.t2[q];
  }
  // 3. Y -= V u on this wave's rows from k on
#pragma unroll
  for (int j = 0; j < kHqRhsRbw; ++j) {
    const int r0 = (wave + kHqRhsWaves * j) * 16;
    __builtin_amdgcn_sched_barrier(0);
    if (j + 1 < kHqRhsRbw) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        vv[(j + 1) & 1][kk] = hq_v_raw(A, M, k, nb, r0 + kHqRhsWaves * 16 + lr, 4 * kk + lq);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (r0 >= M) break;
    if (r0 + 15 < k) continue;
    Cacc d;
    cacc_zero(d);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double2 v = hq_v_mask(vv[j & 1][kk], M, k, nb, r0 + lr, 4 * kk + lq);
      cacc_step(d, v.x, v.y, ur[kk], ui[kk]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      yr[j][q] -= d.t1[q] - d.t2[q];
      yi[j][q] -= d.t3[q] - d.t1[q] - d.t2[q];
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// One workgroup of eight waves per 16 right-hand-side columns of one layer.
// The M x 16 tile Y lives in registers: wave w holds row blocks w + 8 j, lane
// (lq, lr) rows 16 b + lq + 4 q of column lr in register q, which is also
// the B-operand layout of the matrix cores (k-step q), so every product
// below reads Y, w and u where they already are.  Per panel of reflectors V
// (one round of loads, both operand layouts): w = V^H Y, partial sums of the
// waves reduced through LDS (double-buffered, one barrier per panel);
// u = T^H w; Y -= V u.  Then R X = Y(0:c) by 16-row blocks from the bottom
// in LDS: substitution inside each diagonal block (R's diagonal spans the
// Tikhonov scale, so no explicit block inverse), the rows above updated on
// the matrix cores.
template <int kHqRhsRbw>  // row blocks per wave: 3 up to kHqRhsSmallRows rows, 4 up to kHqMaxRows
__device__ __forceinline__ void hq_rhs_body(const HqDesc& D, int tx) {
  const int c = D.c, M = D.m + c;
  const int col0 = tx * kHqRhsCols;
  if (col0 >= D.ncol) return;
  const int nc = min(kHqRhsCols, D.ncol - col0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  const cplx* A = D.A;
  cplx* B = D.A + (size_t)c * M;  // right-hand sides start after the c columns of S
  extern __shared__ double pool[];  // 2 x waves x 2 x 4 x 64 partial sums, then the c x 16 tile
  hvec4 yr[kHqRhsRbw], yi[kHqRhsRbw];
#pragma unroll
  for (int j = 0; j < kHqRhsRbw; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // clamped, not masked: rows past M meet zero reflector rows, columns
      // past nc are not stored; parts loaded straight into the accumulators
      const int r = (wave + kHqRhsWaves * j) * 16 + lq + 4 * q;
      const auto yp = gmem(reinterpret_cast<const double*>(B + (uint32_t)((col0 + min(lr, nc - 1)) * M + min(r, M - 1))));
      yr[j][q] = yp[0];
      yi[j][q] = yp[1];
    }
  const int npan = (c + kHqNb - 1) / kHqNb;
  for (int p = 0; p < npan; ++p) {
    const int k = p * kHqNb;
    hq_apply_panel<kHqRhsRbw>(yr, yi, A, M, k, min(kHqNb, c - k), D.T + (size_t)p * kHqNb * kHqNb,
                              pool + (size_t)(p & 1) * kHqRhsWaves * 2 * 4 * 64);
  }
  // 4. the top c rows into LDS (the partial-sum buffers are done with)
  __syncthreads();
  double2* Ys = reinterpret_cast<double2*>(pool);  // Ys[r * 16 + col]
#pragma unroll
  for (int j = 0; j < kHqRhsRbw; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = (wave + kHqRhsWaves * j) * 16 + lq + 4 * q;
      if (r < c) Ys[r * kHqRhsCols + lr] = make_double2(yr[j][q], yi[j][q]);
    }
  __shared__ double2 Rb[kHqNb][kHqNb + 1];
  for (int b = npan - 1; b >= 0; --b) {
    const int j0 = b * kHqNb;
    const int nbb = min(kHqNb, c - j0);
    {
      const int r = tid % kHqNb, q = tid / kHqNb;
      if (q < kHqNb) Rb[r][q] = (r < nbb && q < nbb && r <= q) ? hld(A + (size_t)(j0 + q) * M + j0 + r)
                                                                : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (wave < kHqRhsCols / 4) {
      // waves 0..3: lane 16 g + i holds row i of column 4 wave + g; row r's
      // value is final at step r and reaches its column's other rows by a
      // DPP broadcast within the row of 16 lanes
      const int col = 4 * wave + (lane >> 4), ri = lane & 15;
      double2 y = ri < nbb ? Ys[(j0 + ri) * kHqRhsCols + col] : make_double2(0.0, 0.0);
      const double2 d = Rb[ri][ri];
      const double dd = d.x * d.x + d.y * d.y;
      const double2 inv = ri < nbb && dd != 0.0 ? make_double2(d.x / dd, -d.y / dd) : make_double2(0.0, 0.0);
#pragma unroll
      for (int r = kHqNb - 1; r >= 0; --r) {
        if (r >= nbb) continue;  // uniform
        const double2 xl = make_double2(y.x * inv.x - y.y * inv.y, y.x * inv.y + y.y * inv.x);
        const double xr = row_bcast16(xl.x, r), xi = row_bcast16(xl.y, r);
        if (ri == r) {
          y = make_double2(xr, xi);
        } else if (ri < r) {
          const double2 a = Rb[ri][r];
          y.x -= a.x * xr - a.y * xi;
          y.y -= a.x * xi + a.y * xr;
        }
      }
      if (ri < nbb) Ys[(j0 + ri) * kHqRhsCols + col] = y;
    }
    __syncthreads();
    double xr[4], xi[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int q = 4 * kk + lq;
      const double2 x = q < nbb ? Ys[(j0 + q) * kHqRhsCols + lr] : make_double2(0.0, 0.0);
      xr[kk] = x.x;
      xi[kk] = x.y;
    }
    for (int r0 = 16 * wave; r0 < j0; r0 += 16 * kHqRhsWaves) {
      Cacc d;
      cacc_zero(d);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int q = 4 * kk + lq;
        const double2 a = q < nbb ? hld(A + (size_t)(j0 + q) * M + r0 + lr) : make_double2(0.0, 0.0);
        cacc_step(d, a.x, a.y, xr[kk], xi[kk]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + lq + 4 * q;
        double2 y = Ys[r * kHqRhsCols + lr];
        y.x -= d.t1[q] - d.t2[q];
        y.y -= d.t3[q] - d.t1[q] - d.t2[q];
        Ys[r * kHqRhsCols + lr] = y;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < c * kHqRhsCols; e += kHqRhsWaves * 64) {
    const int r = e % c, j = e / c;
    if (j < nc) hst(B + (size_t)(col0 + j) * M + r, Ys[r * kHqRhsCols + j]);
  }
}

// Both size classes in one launch: layers [0, n3) (at most kHqRhsSmallRows
// rows, listed first) take three row blocks per wave, the others four, so
// the few large layers do not wait for a launch of their own.
__global__ __launch_bounds__(kHqRhsWaves * 64) void hq_rhs_kernel(const HqDesc* __restrict__ descs, int n3) {
  if ((int)blockIdx.y < n3)
    hq_rhs_body<3>(descs[blockIdx.y], blockIdx.x);
  else
    hq_rhs_body<4>(descs[blockIdx.y], blockIdx.x);
}

// The later columns of S for panel k: Y <- H^H Y on 16 columns per
// workgroup, the tile in registers as in hq_rhs_kernel (rows below k only
// are read back and changed).
template <int kHqRhsRbw>
__device__ __forceinline__ void hq_update_body(const HqDesc& D, int k, int tx) {
  const int c = D.c, M = D.m + c;
  if (k >= c) return;
  const int nb = min(kHqNb, c - k);
  const int c0 = k + nb + tx * kHqRhsCols;
  if (c0 >= c) return;
  const int nc = min(kHqRhsCols, c - c0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  cplx* A = D.A;
  extern __shared__ double pool[];
  hvec4 yr[kHqRhsRbw], yi[kHqRhsRbw];
#pragma unroll
  for (int j = 0; j < kHqRhsRbw; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // clamped, not masked: rows past M meet zero reflector rows, columns
      // past nc are not stored
      const int r = (wave + kHqRhsWaves * j) * 16 + lq + 4 * q;
      const auto yp = gmem(reinterpret_cast<const double*>(A + (uint32_t)((c0 + min(lr, nc - 1)) * M + min(r, M - 1))));
      yr[j][q] = yp[0];
      yi[j][q] = yp[1];
    }
  hq_apply_panel<kHqRhsRbw>(yr, yi, A, M, k, nb, D.T + (size_t)(k / kHqNb) * kHqNb * kHqNb, pool);
  if (lr < nc)
#pragma unroll
    for (int j = 0; j < kHqRhsRbw; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = (wave + kHqRhsWaves * j) * 16 + lq + 4 * q;
        if (r >= k && r < M) hst(A + (uint32_t)((c0 + lr) * M + r), make_double2(yr[j][q], yi[j][q]));
      }
}

// both size classes in one launch, as for hq_rhs_kernel
__global__ __launch_bounds__(kHqRhsWaves * 64) void hq_update_kernel(const HqDesc* __restrict__ descs, int k,
                                                                     int n3) {
  if ((int)blockIdx.y < n3)
    hq_update_body<3>(descs[blockIdx.y], k, blockIdx.x);
  else
    hq_update_body<4>(descs[blockIdx.y], k, blockIdx.x);
}

void launch_hq_prep(const HqDesc* d, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(hq_prep_kernel, dim3(n), dim3(256), 0, st, d);
}
void launch_hq_panel(const HqDesc* d, int n, int k, hipStream_t st, const AsmJob* asm_jobs, int asm_njobs,
                     int asm_t0, int asm_t1) {
  const int extra = asm_t1 > asm_t0 ? (asm_t1 - asm_t0 + kHqPanelThreads / 256 - 1) / (kHqPanelThreads / 256) : 0;
  if (n > 0)
    hipLaunchKernelGGL(hq_panel_kernel, dim3(n + extra), dim3(kHqPanelThreads), 0, st, d, n, k, asm_jobs, asm_njobs,
                       asm_t0, asm_t1);
}
// One launch over both size classes: descs[0, n_small) have at most
// kHqRhsSmallRows rows and take three row blocks per wave (unless
// row_blocks is 4), descs[n_small, n_small + n_large) take four.
void launch_hq_update(const HqDesc* d, int n_small, int n_large, int k, int max_c, hipStream_t st, int row_blocks) {
  const int tiles = (max_c - k - kHqNb + kHqRhsCols - 1) / kHqRhsCols;
  const size_t red = sizeof(double) * kHqRhsWaves * 2 * 4 * 64;
  const int n = n_small + n_large;
  if (n <= 0 || tiles <= 0) return;
  hipLaunchKernelGGL(hq_update_kernel, dim3(tiles, n), dim3(kHqRhsWaves * 64), red, st, d, k,
                     row_blocks == 3 ? n_small : 0);
}
void launch_hq_rhs(const HqDesc* d, int n_small, int n_large, int max_ncol, int max_c, hipStream_t st,
                   int row_blocks) {
  const int tiles = (max_ncol + kHqRhsCols - 1) / kHqRhsCols;
  const size_t red = sizeof(double) * 2 * kHqRhsWaves * 2 * 4 * 64;
  const size_t tile = sizeof(double2) * (size_t)max_c * kHqRhsCols;
  const int n = n_small + n_large;
  if (n <= 0 || tiles <= 0) return;
  hipLaunchKernelGGL(hq_rhs_kernel, dim3(tiles, n), dim3(kHqRhsWaves * 64), std::max(red, tile), st, d,
                     row_blocks == 3 ? n_small : 0);
}

}  // namespace mlh

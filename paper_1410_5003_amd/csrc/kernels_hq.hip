// Blocked Householder least squares for the per-layer Schur eliminations
// (Sec. 3.2: the products Q^+ C are obtained from a backward-stable dense
// least-squares solve, never from an explicit pseudo-inverse).  The problem
// solved is the Tikhonov-stacked one, min ||Q X - C||^2 + mu^2 ||X||^2,
// i.e. the QR factorisation of [Q; mu I] applied to [C; 0].
//
//   hq_prep_kernel     mu = mu_rel ||Q||_F and the mu I rows;
//   hq_panel_kernel    Householder QR of a 16-column panel in LDS, and the
//                      triangular factor T of its block reflector
//                      H = I - V T V^H (compact WY form);
//   hq_update_kernel   the later columns of S: Y <- H^H Y = Y - V T^H (V^H Y),
//                      32 columns per workgroup, one wavefront per column;
//   hq_rhs_kernel      after the last panel, one workgroup per 16 right-hand
//                      sides: the (M x 16) tile stays in LDS while every block
//                      reflector is applied to it and R X = (Q^H C)[0:c] is
//                      solved by 16-row blocks (substitution inside each
//                      diagonal block, products on the FP64 matrix cores
//                      elsewhere).  The right-hand sides cross HBM once
//                      instead of once per panel.
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

// Panel rows k..M-1 of columns k..k+15 in LDS (stride 17 against bank
// conflicts).  Thread (j, q) = (tid / 16, tid % 16) owns column j of the rows
// congruent to q modulo 16 below the current reflector, so each column step
// is one pass (the norm of column i and the raw products of column i with
// the later columns), sums over the 16 lanes of a DPP row, one barrier, and
// one update pass.  The scaling of column i into its Householder vector is
// deferred to the next pass, which does not read that column.
__global__ __launch_bounds__(256) void hq_panel_kernel(const HqDesc* __restrict__ descs, int k) {
  const HqDesc& D = descs[blockIdx.x];
  const int c = D.c, M = D.m + c;
  if (k >= c) return;
  const int nb = min(kHqNb, c - k);
  const int L = M - k;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int jc = tid >> 4, q16 = tid & 15;
  __shared__ double2 pan[kHqMaxRows][kHqNb + 1];
  __shared__ double2 red[2][kHqNb];
  __shared__ double2 tau[kHqNb], scl[kHqNb];
  __shared__ double2 gram[kHqNb][kHqNb + 1];
  __shared__ double2 T[kHqNb][kHqNb + 1];
  cplx* A = D.A;
  for (int e = tid; e < L * kHqNb; e += 256) {
    const int r = e % L, j = e / L;
    pan[r][j] = j < nb ? hld(A + (size_t)(k + j) * M + k + r) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    const int buf = i & 1;
    // deferred: column i - 1 becomes its Householder vector
    if (i > 0 && jc == i - 1) {
      const double2 sc = scl[i - 1];
      for (int r = i + q16; r < L; r += 16) {
        const double2 x = pan[r][i - 1];
        pan[r][i - 1] = make_double2(x.x * sc.x - x.y * sc.y, x.x * sc.y + x.y * sc.x);
      }
    }
    // pass 1: |x|^2 below the diagonal of column i; raw products of column i
    // with the later columns (rows below i)
    double ar = 0.0, ai = 0.0;
    if (jc >= i) {
#pragma unroll 4
      for (int r = i + 1 + q16; r < L; r += 16) {
        const double2 x = pan[r][i];
        if (jc == i) {
          ar += x.x * x.x + x.y * x.y;
        } else {
          const double2 y = pan[r][jc];
          ar += x.x * y.x + x.y * y.y;  // conj(x) y
          ai += x.x * y.y - x.y * y.x;
        }
      }
    }
    ar = row16_sum(ar);
    ai = row16_sum(ai);
    if (q16 == 15) red[buf][jc] = make_double2(ar, ai);
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
      if (q16 == 0) pan[i][jc] = make_double2(yi.x - ur, yi.y - ui);
#pragma unroll 4
      for (int r = i + 1 + q16; r < L; r += 16) {
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
    for (int r = nb + q16; r < L; r += 16) {
      const double2 x = pan[r][nb - 1];
      pan[r][nb - 1] = make_double2(x.x * sc.x - x.y * sc.y, x.x * sc.y + x.y * sc.x);
    }
  }
  __syncthreads();
  // Gram matrix G = V^H V (V unit lower trapezoidal): thread (b, q) sums
  // conj(v_a) v_b over its rows for every a < b
  {
    double2 g[kHqNb];
#pragma unroll
    for (int a = 0; a < kHqNb; ++a) g[a] = make_double2(0.0, 0.0);
    if (jc < nb) {
#pragma unroll 4
      for (int r = jc + q16; r < L; r += 16) {
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
    }
#pragma unroll
    for (int a = 0; a < kHqNb; ++a) {
      const double gr = row16_sum(g[a].x), gi = row16_sum(g[a].y);
      if (q16 == 15 && a < jc && jc < nb) gram[a][jc] = make_double2(gr, gi);
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
  for (int e = tid; e < kHqNb * kHqNb; e += 256) hst(D.T + (size_t)pidx * kHqNb * kHqNb + e, T[e % kHqNb][e / kHqNb]);
  for (int e = tid; e < L * nb; e += 256) {
    const int r = e % L, j = e / L;
    hst(A + (size_t)(k + j) * M + k + r, pan[r][j]);
  }
}

// Y <- Y - V (T^H (V^H Y)) for 32 columns: one wavefront per column, lanes
// over rows; V (rows k..M-1, unit diagonal implicit) staged in LDS
__global__ __launch_bounds__(256) void hq_update_kernel(const HqDesc* __restrict__ descs, int k) {
  const HqDesc& D = descs[blockIdx.y];
  const int c = D.c, M = D.m + c;
  if (k >= c) return;
  const int nb = min(kHqNb, c - k);
  const int L = M - k;
  const int total = c;  // right-hand sides: hq_rhs_kernel
  const int c0 = k + nb + blockIdx.x * kHqCols;
  if (c0 >= total) return;
  const int nc = min(kHqCols, total - c0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double2 V[kHqMaxRows][kHqNb + 1];
  __shared__ double2 T[kHqNb][kHqNb + 1];
  cplx* A = D.A;
  for (int e = tid; e < L * kHqNb; e += 256) {
    const int r = e % L, j = e / L;
    double2 v = make_double2(0.0, 0.0);
    if (j < nb) {
      if (r == j)
        v = make_double2(1.0, 0.0);
      else if (r > j)
        v = hld(A + (size_t)(k + j) * M + k + r);
    }
    V[r][j] = v;
  }
  const cplx* Tk = D.T + (size_t)(k / kHqNb) * kHqNb * kHqNb;  // this panel's T
  for (int e = tid; e < kHqNb * kHqNb; e += 256) T[e % kHqNb][e / kHqNb] = hld(Tk + e);
  __syncthreads();
  __shared__ double2 wsh[4][kHqNb], ush[4][kHqNb];
  for (int cc = wave; cc < nc; cc += 4) {
    cplx* y = A + (size_t)(c0 + cc) * M + k;
    // w = V^H y  (16 partial sums per lane, then a wavefront reduction)
    double2 w[kHqNb];
#pragma unroll
    for (int i = 0; i < kHqNb; ++i) w[i] = make_double2(0.0, 0.0);
    for (int r = lane; r < L; r += 64) {
      const double2 b = hld(y + r);
#pragma unroll
      for (int i = 0; i < kHqNb; ++i) {
        const double2 v = V[r][i];
        w[i].x += v.x * b.x + v.y * b.y;
        w[i].y += v.x * b.y - v.y * b.x;
      }
    }
#pragma unroll
    for (int i = 0; i < kHqNb; ++i) {
      const double a = hwave_sum(w[i].x), b = hwave_sum(w[i].y);
      if (lane == i) wsh[wave][i] = make_double2(a, b);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // u = T^H w
    if (lane < kHqNb) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < kHqNb; ++q) {
        const double2 t = T[q][lane], x = wsh[wave][q];  // conj(T[q][i]) w[q]
        sr += t.x * x.x + t.y * x.y;
        si += t.x * x.y - t.y * x.x;
      }
      ush[wave][lane] = make_double2(sr, si);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // y -= V u
    for (int r = lane; r < L; r += 64) {
      double2 b = hld(y + r);
#pragma unroll
      for (int i = 0; i < kHqNb; ++i) {
        const double2 v = V[r][i], u = ush[wave][i];
        b.x -= v.x * u.x - v.y * u.y;
        b.y -= v.x * u.y + v.y * u.x;
      }
      hst(y + r, b);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

typedef double hvec4 __attribute__((ext_vector_type(4)));

// V of panel k as an MFMA operand value: column i, row r (global); unit
// diagonal and zeros above it, Householder vectors below
__device__ inline double2 hq_v(const cplx* A, int M, int k, int nb, int r, int i) {
  if (i >= nb || r < k + i) return make_double2(0.0, 0.0);
  if (r == k + i) return make_double2(1.0, 0.0);
  return hld(A + (size_t)(k + i) * M + r);
}

constexpr int kHqRhsCols = 16;
constexpr int kHqRhsWaves = 4;

__global__ __launch_bounds__(kHqRhsWaves * 64) void hq_rhs_kernel(const HqDesc* __restrict__ descs) {
  const HqDesc& D = descs[blockIdx.y];
  const int c = D.c, M = D.m + c;
  const int col0 = blockIdx.x * kHqRhsCols;
  if (col0 >= D.ncol) return;
  const int nc = min(kHqRhsCols, D.ncol - col0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  const cplx* A = D.A;
  cplx* B = D.A + (size_t)c * M;  // right-hand sides start after the c columns of S
  __shared__ double2 Y[kHqMaxRows][kHqRhsCols];
  __shared__ double red[kHqRhsWaves][2][4][64];
  for (int e = tid; e < M * kHqRhsCols; e += kHqRhsWaves * 64) {
    const int r = e % M, j = e / M;
    Y[r][j] = j < nc ? hld(B + (size_t)(col0 + j) * M + r) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int npan = (c + kHqNb - 1) / kHqNb;
  for (int p = 0; p < npan; ++p) {
    const int k = p * kHqNb;
    const int nb = min(kHqNb, c - k);
    const cplx* Tp = D.T + (size_t)p * kHqNb * kHqNb;
    // 1. partial w = V^H Y over this wave's 4-row steps of rows k..M-1
    hvec4 wr = {0, 0, 0, 0}, wi = {0, 0, 0, 0};
    // four 4-row steps per batch, all loads issued before the products
    for (int r0 = k + 4 * wave; r0 < M; r0 += 16 * kHqRhsWaves) {
      double2 v[4], y[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int r = r0 + 4 * kHqRhsWaves * b + lq;
        v[b] = r < M ? hq_v(A, M, k, nb, r, lr) : make_double2(0.0, 0.0);  // A[i=lr][k=r]
        y[b] = r < M ? Y[r][lr] : make_double2(0.0, 0.0);                  // B[k=r][col=lr]
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {  // w = conj(V)^T Y
        wr = __builtin_amdgcn_mfma_f64_16x16x4f64(v[b].x, y[b].x, wr, 0, 0, 0);
        wr = __builtin_amdgcn_mfma_f64_16x16x4f64(v[b].y, y[b].y, wr, 0, 0, 0);
        wi = __builtin_amdgcn_mfma_f64_16x16x4f64(v[b].x, y[b].y, wi, 0, 0, 0);
        wi = __builtin_amdgcn_mfma_f64_16x16x4f64(-v[b].y, y[b].x, wi, 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      red[wave][0][q][lane] = wr[q];
      red[wave][1][q][lane] = wi[q];
    }
    __syncthreads();
    // 2. full w in every wave (register q: row 4q + lq, column lr), then
    //    u = T^H w on the matrix cores (the result is again in that layout)
    double w_r[4], w_i[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int w = 0; w < kHqRhsWaves; ++w) {
        a += red[w][0][q][lane];
        b += red[w][1][q][lane];
      }
      w_r[q] = a;
      w_i[q] = b;
    }
    hvec4 ur = {0, 0, 0, 0}, ui = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int q = 4 * kk + lq;
      const double2 t = hld(Tp + (size_t)lr * kHqNb + q);  // T[q][i = lr]; A = conj(T)^T
      ur = __builtin_amdgcn_mfma_f64_16x16x4f64(t.x, w_r[kk], ur, 0, 0, 0);
      ur = __builtin_amdgcn_mfma_f64_16x16x4f64(t.y, w_i[kk], ur, 0, 0, 0);
      ui = __builtin_amdgcn_mfma_f64_16x16x4f64(t.x, w_i[kk], ui, 0, 0, 0);
      ui = __builtin_amdgcn_mfma_f64_16x16x4f64(-t.y, w_r[kk], ui, 0, 0, 0);
    }
    // 3. Y(rows k..M-1) -= V u, 16-row blocks (k is a multiple of 16)
    for (int r0 = k + 16 * wave; r0 < M; r0 += 16 * kHqRhsWaves) {
      hvec4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};
      double2 v[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int i = 4 * kk + lq, r = r0 + lr;
        v[kk] = r < M ? hq_v(A, M, k, nb, r, i) : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        ar = __builtin_amdgcn_mfma_f64_16x16x4f64(v[kk].x, ur[kk], ar, 0, 0, 0);
        ar = __builtin_amdgcn_mfma_f64_16x16x4f64(-v[kk].y, ui[kk], ar, 0, 0, 0);
        ai = __builtin_amdgcn_mfma_f64_16x16x4f64(v[kk].x, ui[kk], ai, 0, 0, 0);
        ai = __builtin_amdgcn_mfma_f64_16x16x4f64(v[kk].y, ur[kk], ai, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + lq + 4 * q;
        if (r < M) {
          double2 y = Y[r][lr];
          y.x -= ar[q];
          y.y -= ai[q];
          Y[r][lr] = y;
        }
      }
    }
    __syncthreads();
  }
  // 4. R X = Y(0:c) by 16-row blocks from the bottom: substitution inside
  //    the diagonal block (one thread per column; R's diagonal spans the
  //    Tikhonov scale, so no explicit block inverse), then
  //    Y(rows above) -= R(rows above, block) X_b on the matrix cores
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
    if (tid < kHqRhsCols) {
      for (int r = nbb - 1; r >= 0; --r) {
        double2 acc = Y[j0 + r][tid];
        for (int q = r + 1; q < nbb; ++q) {
          const double2 a = Rb[r][q], x = Y[j0 + q][tid];
          acc.x -= a.x * x.x - a.y * x.y;
          acc.y -= a.x * x.y + a.y * x.x;
        }
        const double2 d = Rb[r][r];
        const double dd = d.x * d.x + d.y * d.y;
        Y[j0 + r][tid] = make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd);
      }
    }
    __syncthreads();
    double xr[4], xi[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int q = 4 * kk + lq;
      const double2 x = q < nbb ? Y[j0 + q][lr] : make_double2(0.0, 0.0);
      xr[kk] = x.x;
      xi[kk] = x.y;
    }
    for (int r0 = 16 * wave; r0 < j0; r0 += 16 * kHqRhsWaves) {
      hvec4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int q = 4 * kk + lq;
        const double2 a = q < nbb ? hld(A + (size_t)(j0 + q) * M + r0 + lr) : make_double2(0.0, 0.0);
        ar = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, xr[kk], ar, 0, 0, 0);
        ar = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, xi[kk], ar, 0, 0, 0);
        ai = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, xi[kk], ai, 0, 0, 0);
        ai = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, xr[kk], ai, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + lq + 4 * q;
        double2 y = Y[r][lr];
        y.x -= ar[q];
        y.y -= ai[q];
        Y[r][lr] = y;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < c * kHqRhsCols; e += kHqRhsWaves * 64) {
    const int r = e % c, j = e / c;
    if (j < nc) hst(B + (size_t)(col0 + j) * M + r, Y[r][j]);
  }
}

void launch_hq_prep(const HqDesc* d, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(hq_prep_kernel, dim3(n), dim3(256), 0, st, d);
}
void launch_hq_panel(const HqDesc* d, int n, int k, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(hq_panel_kernel, dim3(n), dim3(256), 0, st, d, k);
}
void launch_hq_update(const HqDesc* d, int n, int k, int max_cols, hipStream_t st) {
  const int tiles = (max_cols - k - 1) / kHqCols + 1;
  if (n > 0 && tiles > 0) hipLaunchKernelGGL(hq_update_kernel, dim3(tiles, n), dim3(256), 0, st, d, k);
}
void launch_hq_rhs(const HqDesc* d, int n, int max_ncol, hipStream_t st) {
  const int tiles = (max_ncol + kHqRhsCols - 1) / kHqRhsCols;
  if (n > 0 && tiles > 0)
    hipLaunchKernelGGL(hq_rhs_kernel, dim3(tiles, n), dim3(kHqRhsWaves * 64), 0, st, d);
}

}  // namespace mlh

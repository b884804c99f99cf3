// Batched blocked Gauss-Jordan elimination with partial pivoting for the
// block-tridiagonal sweep (Sec. 3.3).  Each sweep step needs
// [U_i | g_i] = A~_ii^{-1} [A'_{i,i+1} | f~_i]; the diagonal blocks come from a
// second-kind equation and are well conditioned, so applying their inverse
// (rather than back-substituting with LU factors) is accurate, and it turns
// the whole step into one panel-by-panel elimination whose bulk is a
// matrix-core product.
//
// Panel step k (columns k..k+NB-1), for every matrix of the batch:
//   gje_panel_kernel   one workgroup: LU with partial pivoting of the tall
//                      panel rows k..n-1 held in registers; writes the row
//                      interchanges, applies them to the panel columns of W
//                      and writes the inverse M1 of the NB x NB pivot block.
//                      The multipliers of the update are the panel values
//                      themselves (original values for rows >= k, current
//                      values above k), read from W;
//   gje_update_kernel  one workgroup per 32 trailing columns of the diagonal
//                      block: applies the row swaps, Z = M1 Y(pivot rows),
//                      Y(other rows) -= P Z on the FP64 matrix cores,
//                      Y(pivot rows) = Z.
//   gje_rhs_kernel     after the last step: one workgroup per 16 (8 for
//                      n > 608) right-hand-side columns keeps its tile in LDS and applies
//                      every step's interchanges and update to it, reading the
//                      multipliers P (the panel columns of W, unchanged after
//                      their step) and M1 of each step.  The right-hand sides
//                      thus cross HBM once instead of once per step.
#include <algorithm>

#include "internal.hpp"

namespace mlh {

typedef double dvec4 __attribute__((ext_vector_type(4)));

__device__ inline double2 gld(const cplx* p) { return *reinterpret_cast<const double2*>(p); }
__device__ inline void gst(cplx* p, double2 v) { *reinterpret_cast<double2*>(p) = v; }
__device__ inline double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cinv2(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

// Panel kernel: the n x NB panel columns live in registers, thread t owning
// rows t and t + 512.  The kernel first applies the previous step's
// transformation to them (the update kernel does the other columns), then
// factors rows k..n-1.  Rows are not moved while the panel is
// factored: a row that wins the pivot search for column c is marked done and
// broadcast through LDS, so each column costs one workgroup barrier.  Every
// wave reduces its candidates to one 64-bit key (high word of |a|^2, then the
// complemented row index, so that ties go to the lowest row) with DPP moves,
// and its winning lane stages its row in LDS next to the key.
constexpr int kPanelThreads = 512;
constexpr int kUpdThreads = 1024;
constexpr int kUpdWaves = kUpdThreads / 64;
constexpr int kPanelSlots = (kGjeMaxN + kPanelThreads - 1) / kPanelThreads;
constexpr int kPanelWaves = kPanelThreads / 64;

template <int CTRL, int ROWS>
__device__ inline uint64_t key_max_dpp(uint64_t x) {
  const int lo = (int)(uint32_t)x, hi = (int)(uint32_t)(x >> 32);
  const uint32_t lo2 = (uint32_t)__builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xf, true);
  const uint32_t hi2 = (uint32_t)__builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xf, true);
  const uint64_t y = ((uint64_t)hi2 << 32) | lo2;
  return y > x ? y : x;
}

// maximum of x over the wavefront, returned in every lane
__device__ inline uint64_t wave_key_max(uint64_t x) {
  x = key_max_dpp<0x111, 0xf>(x);  // row_shr:1
  x = key_max_dpp<0x112, 0xf>(x);  // row_shr:2
  x = key_max_dpp<0x114, 0xf>(x);  // row_shr:4
  x = key_max_dpp<0x118, 0xf>(x);  // row_shr:8  -> lane 15 of each row: row maximum
  x = key_max_dpp<0x142, 0xa>(x);  // row_bcast:15 into rows 1, 3
  x = key_max_dpp<0x143, 0xc>(x);  // row_bcast:31 into rows 2, 3 -> lane 63: wave maximum
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t pivot_key(double2 v, int lr) {
  const double m2 = v.x * v.x + v.y * v.y;
  const uint64_t hi = (uint64_t)(__double_as_longlong(m2)) >> 32;  // monotone for m2 >= 0
  return (hi << 32) | (uint64_t)(0xffffffffu - (uint32_t)lr);
}

// state of one panel factorisation shared by the per-column steps
struct PanelState {
  double2 a[kPanelSlots][kGjeNb];
  int pidx[kPanelSlots];  // pivot order of the row, -1 while still eligible
  int singular;
};

struct PanelShared {
  uint64_t key[2][kPanelWaves];
  double2 row[2][kPanelWaves][kGjeNb];
  int spiv[kGjeNb];
};

// one column of the panel LU; C is a template parameter so that every
// register index is static
template <int C>
__device__ __forceinline__ void panel_column(PanelState& st, PanelShared& sh, int nb, int k, int tid) {
  if (C >= nb) return;
  const int lane = tid & 63, wave = tid >> 6;
  const int buf = C & 1;
  uint64_t best = 0;
#pragma unroll
  for (int sl = 0; sl < kPanelSlots; ++sl) {
    const uint64_t key = st.pidx[sl] < 0 ? pivot_key(st.a[sl][C], tid + sl * kPanelThreads) : 0;
    best = key > best ? key : best;
  }
  const uint64_t wbest = wave_key_max(best);
  if (lane == 0) sh.key[buf][wave] = wbest;
  if (wbest != 0 && best == wbest) {  // this lane holds the wave's candidate row
    const int sl = (int)(0xffffffffu - (uint32_t)wbest) / kPanelThreads;
#pragma unroll
    for (int s2 = 0; s2 < kPanelSlots; ++s2)
      if (s2 == sl)
#pragma unroll
        for (int j = 0; j < kGjeNb; ++j) sh.row[buf][wave][j] = st.a[s2][j];
  }
  __syncthreads();
  uint64_t kb = sh.key[buf][0];
  int wb = 0;
#pragma unroll
  for (int w = 1; w < kPanelWaves; ++w) {
    const uint64_t kw = sh.key[buf][w];
    if (kw > kb) {
      kb = kw;
      wb = w;
    }
  }
  const int p = (int)(0xffffffffu - (uint32_t)kb);
  if ((kb >> 32) == 0 && st.singular == 0) st.singular = k + C + 1;
  if (tid == 0) sh.spiv[C] = p;
  const double2 ucc = sh.row[buf][wb][C];
  const bool ok = (ucc.x != 0.0 || ucc.y != 0.0);
  const double2 ip = ok ? cinv2(ucc) : make_double2(0.0, 0.0);
  double2 prow[kGjeNb];
#pragma unroll
  for (int j = C + 1; j < kGjeNb; ++j) prow[j] = sh.row[buf][wb][j];
#pragma unroll
  for (int sl = 0; sl < kPanelSlots; ++sl) {
    const int lr = tid + sl * kPanelThreads;
    if (lr == p) {
      st.pidx[sl] = C;
    } else if (st.pidx[sl] < 0) {
      const double2 l = cmul2(st.a[sl][C], ip);
      st.a[sl][C] = l;
#pragma unroll
      for (int j = C + 1; j < kGjeNb; ++j) {
        const double2 t = cmul2(l, prow[j]);
        st.a[sl][j].x -= t.x;
        st.a[sl][j].y -= t.y;
      }
    }
  }
}

template <int C>
struct PanelColumns {
  static __device__ __forceinline__ void run(PanelState& st, PanelShared& sh, int nb, int k, int tid) {
    panel_column<C>(st, sh, nb, k, tid);
    PanelColumns<C + 1>::run(st, sh, nb, k, tid);
  }
};
template <>
struct PanelColumns<kGjeNb> {
  static __device__ __forceinline__ void run(PanelState&, PanelShared&, int, int, int) {}
};

__global__ __launch_bounds__(kPanelThreads) void gje_panel_kernel(const GjeDesc* __restrict__ descs, int k) {
  const GjeDesc& D = descs[blockIdx.x];
  const int n = D.n;
  if (k >= n) return;
  const int nb = min(kGjeNb, n - k);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  cplx* W = D.W;
  __shared__ PanelShared sh;
  __shared__ double2 lu11[kGjeNb][kGjeNb + 1];
  __shared__ int sdst[2 * kGjeNb], ssrc[2 * kGjeNb], snaff;
  __shared__ double2 stage[2 * kGjeNb][kGjeNb];
  __shared__ double2 zs[kGjeNb][kGjeNb];
  if (k > 0) {
    // the previous step's transformation on these 16 columns, in W (the
    // update kernel does the columns after them): its row interchanges,
    // Z = M1 Y(its pivot rows) and Y(other rows) -= P Z on the matrix cores
    const int kp = k - kGjeNb;
    const int lr = lane & 15, lq = lane >> 4;
    const int* pivp = D.piv + (size_t)(kp / kGjeNb) * kGjePivStride;
    const cplx* M1p = D.M1 + (size_t)(kp / kGjeNb) * kGjeNb * kGjeNb;
    if (tid == 0) snaff = pivp[0];
    if (tid < 2 * kGjeNb) {
      sdst[tid] = pivp[1 + tid];
      ssrc[tid] = pivp[1 + 2 * kGjeNb + tid];
    }
    __syncthreads();
    const int nap = snaff;
    for (int e = tid; e < nap * kGjeNb; e += kPanelThreads) {
      const int t = e % nap, j = e / nap;
      stage[t][j] = j < nb ? gld(W + (size_t)(k + j) * n + ssrc[t]) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int e = tid; e < nap * kGjeNb; e += kPanelThreads) {
      const int t = e % nap, j = e / nap;
      if (j < nb) gst(W + (size_t)(k + j) * n + sdst[t], stage[t][j]);
    }
    __syncthreads();
    if (wave == 0) {  // Z = M1 Y1: lane holds M1[lr][q] and Y1[q][lr], q = 4 kk + lq
      dvec4 zr = {0, 0, 0, 0}, zi = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int q = 4 * kk + lq;
        const double2 m = gld(M1p + (size_t)q * kGjeNb + lr);
        const double2 y = lr < nb ? gld(W + (size_t)(k + lr) * n + kp + q) : make_double2(0.0, 0.0);
        zr = __builtin_amdgcn_mfma_f64_16x16x4f64(m.x, y.x, zr, 0, 0, 0);
        zr = __builtin_amdgcn_mfma_f64_16x16x4f64(-m.y, y.y, zr, 0, 0, 0);
        zi = __builtin_amdgcn_mfma_f64_16x16x4f64(m.x, y.y, zi, 0, 0, 0);
        zi = __builtin_amdgcn_mfma_f64_16x16x4f64(m.y, y.x, zi, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) zs[lq + 4 * q][lr] = make_double2(zr[q], zi[q]);
    }
    __syncthreads();
    const int nrb = (n + 15) / 16;
    for (int rb = wave; rb < nrb; rb += kPanelWaves) {
      const int r0 = rb * 16;
      if (r0 == kp) {  // the previous pivot rows receive Z
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (lr < nb) gst(W + (size_t)(k + lr) * n + kp + lq + 4 * q, zs[lq + 4 * q][lr]);
        continue;
      }
      dvec4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int row = r0 + lr, q = 4 * kk + lq;
        const double2 a = row < n ? gld(W + (size_t)(kp + q) * n + row) : make_double2(0.0, 0.0);
        const double2 b = zs[q][lr];
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, acci, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = r0 + lq + 4 * q;
        if (row < n && lr < nb) {
          cplx* p = W + (size_t)(k + lr) * n + row;
          double2 v = gld(p);
          v.x -= accr[q];
          v.y -= acci[q];
          gst(p, v);
        }
      }
    }
    __syncthreads();
  }
  PanelState st;
  st.singular = 0;
  // every row of the panel columns: thread t holds rows t and t + 512
#pragma unroll
  for (int sl = 0; sl < kPanelSlots; ++sl) {
    const int r = tid + sl * kPanelThreads;
    st.pidx[sl] = (r >= k && r < n) ? -1 : kGjeNb;
#pragma unroll
    for (int j = 0; j < kGjeNb; ++j)
      st.a[sl][j] = (r < n && j < nb) ? gld(W + (size_t)(k + j) * n + r) : make_double2(0.0, 0.0);
  }
  double2 (&a)[kPanelSlots][kGjeNb] = st.a;
  int (&pidx)[kPanelSlots] = st.pidx;
  PanelColumns<0>::run(st, sh, nb, k, tid);
  const int singular = st.singular;
  int* spiv = sh.spiv;
  if (tid == 0 && singular != 0) atomicCAS(D.info, 0, singular);
  // the factored pivot block: row of pivot c holds L11 (j < c) and U11 (j >= c)
#pragma unroll
  for (int sl = 0; sl < kPanelSlots; ++sl)
    if (pidx[sl] >= 0 && pidx[sl] < kGjeNb)
#pragma unroll
      for (int j = 0; j < kGjeNb; ++j) lu11[pidx[sl]][j] = a[sl][j];
  if (tid >= nb && tid < kGjeNb)
#pragma unroll
    for (int j = 0; j < kGjeNb; ++j) lu11[tid][j] = make_double2(0.0, 0.0);
  // the row permutation of this step as (destination, source) pairs of
  // global rows: pivot q (row spiv[q], never moved in registers) goes to
  // position k + q; rows of positions k..k+nb-1 that were not chosen fill the
  // positions the chosen rows vacated below the block.  piv[0] = count,
  // piv[1..] destinations, piv[1+2NB..] sources.
  __syncthreads();
  if (tid == 0) {
    int na = 0;
    bool chosen[kGjeNb];
    for (int q = 0; q < kGjeNb; ++q) chosen[q] = false;
    for (int q = 0; q < nb; ++q)
      if (spiv[q] - k < nb) chosen[spiv[q] - k] = true;
    int nxt = 0;  // next pivot row from below the block, in pivot order
    for (int q = 0; q < nb; ++q) {
      if (spiv[q] != k + q) {
        sdst[na] = k + q;
        ssrc[na] = spiv[q];
        ++na;
      }
      if (!chosen[q]) {  // row at position q was displaced: send it below
        while (spiv[nxt] - k < nb) ++nxt;
        sdst[na] = spiv[nxt];
        ssrc[na] = k + q;
        ++na;
        ++nxt;
      }
    }
    int* piv = D.piv + (size_t)(k / kGjeNb) * kGjePivStride;
    piv[0] = na;
    snaff = na;
    for (int t = 0; t < na; ++t) {
      piv[1 + t] = sdst[t];
      piv[1 + 2 * kGjeNb + t] = ssrc[t];
    }
  }
  __syncthreads();
  // apply the interchanges to the panel columns of W, which hold the values
  // the panel started from: the update kernels read their multipliers
  // (those values, for the rows off the pivot block) from there
  const int naff = snaff;
  for (int e = tid; e < naff * kGjeNb; e += kPanelThreads) {
    const int t = e % naff, j = e / naff;
    stage[t][j] = j < nb ? gld(W + (size_t)(k + j) * n + ssrc[t]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int e = tid; e < naff * kGjeNb; e += kPanelThreads) {
    const int t = e % naff, j = e / naff;
    if (j < nb) gst(W + (size_t)(k + j) * n + sdst[t], stage[t][j]);
  }
  // M1 = (L11 U11)^{-1} in wave 0: lane (lq, lr) holds rows lq + 4 q of
  // column lr; X = L11^{-1} by row operations, then M1 = U11^{-1} X
  if (wave == 0) {
    const int lr = lane & 15, lq = lane >> 4;
    double2 x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = make_double2(lq + 4 * q == lr ? 1.0 : 0.0, 0.0);
#pragma unroll
    for (int r = 0; r < kGjeNb - 1; ++r) {
      const double2 xr = make_double2(__shfl(x[r / 4].x, (r % 4) * 16 + lr, 64), __shfl(x[r / 4].y, (r % 4) * 16 + lr, 64));
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lq + 4 * q;
        if (i > r) {
          const double2 l = lu11[i][r];
          x[q].x -= l.x * xr.x - l.y * xr.y;
          x[q].y -= l.x * xr.y + l.y * xr.x;
        }
      }
    }
#pragma unroll
    for (int r = kGjeNb - 1; r >= 0; --r) {
      const double2 d = lu11[r][r];
      const bool ok = r < nb && (d.x != 0.0 || d.y != 0.0);
      double2 xr = make_double2(__shfl(x[r / 4].x, (r % 4) * 16 + lr, 64), __shfl(x[r / 4].y, (r % 4) * 16 + lr, 64));
      xr = ok ? cmul2(xr, cinv2(d)) : make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lq + 4 * q;
        if (i == r) {
          x[q] = xr;
        } else if (i < r) {
          const double2 u = lu11[i][r];
          x[q].x -= u.x * xr.x - u.y * xr.y;
          x[q].y -= u.x * xr.y + u.y * xr.x;
        }
      }
    }
    cplx* M1 = D.M1 + (size_t)(k / kGjeNb) * kGjeNb * kGjeNb;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      gst(M1 + (size_t)lr * kGjeNb + lq + 4 * q, lr < nb ? x[q] : make_double2(0.0, 0.0));
  }
}

// columns [k + nb + lo, min(n, k + nb + hi)) of the diagonal block; the
// right-hand-side columns are left to gje_rhs_kernel, after all steps
__global__ __launch_bounds__(kUpdThreads) void gje_update_kernel(const GjeDesc* __restrict__ descs, int k, int lo,
                                                                 int hi) {
  const GjeDesc& D = descs[blockIdx.y];
  const int n = D.n;
  if (k >= n) return;
  const int nb = min(kGjeNb, n - k);
  const int cend = min(n, k + nb + hi);
  const int c0 = k + nb + lo + blockIdx.x * kGjeCols;
  if (c0 >= cend) return;
  const int nc = min(kGjeCols, cend - c0);
  const int* piv = D.piv + (size_t)(k / kGjeNb) * kGjePivStride;
  const cplx* M1 = D.M1 + (size_t)(k / kGjeNb) * kGjeNb * kGjeNb;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  cplx* W = D.W;
  __shared__ double zr[kGjeNb][kGjeCols + 1], zi[kGjeNb][kGjeCols + 1];
  __shared__ double2 m1[kGjeNb][kGjeNb];
  __shared__ double2 y1[kGjeNb][kGjeCols];
  // 1. row interchanges of this step on our columns, as (destination, source)
  //    pairs composed by the panel kernel: stage the sources, then write back
  __shared__ int sdst[2 * kGjeNb], ssrc[2 * kGjeNb];
  __shared__ double2 stage[2 * kGjeNb][kGjeCols];
  const int naff = piv[0];
  if (tid < naff) {
    sdst[tid] = piv[1 + tid];
    ssrc[tid] = piv[1 + 2 * kGjeNb + tid];
  }
  for (int e = tid; e < kGjeNb * kGjeNb; e += kUpdThreads) m1[e % kGjeNb][e / kGjeNb] = gld(M1 + e);
  __syncthreads();
  for (int e = tid; e < naff * nc; e += kUpdThreads) {
    const int t = e % naff, c = e / naff;
    stage[t][c] = gld(W + (size_t)(c0 + c) * n + ssrc[t]);
  }
  __syncthreads();
  for (int e = tid; e < naff * nc; e += kUpdThreads) {
    const int t = e % naff, c = e / naff;
    gst(W + (size_t)(c0 + c) * n + sdst[t], stage[t][c]);
  }
  __syncthreads();
  // 2. Z = M1 Y1
  for (int e = tid; e < kGjeNb * kGjeCols; e += kUpdThreads) {
    const int r = e % kGjeNb, c = e / kGjeNb;
    y1[r][c] = (r < nb && c < nc) ? gld(W + (size_t)(c0 + c) * n + k + r) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int e = tid; e < kGjeNb * kGjeCols; e += kUpdThreads) {
    const int r = e % kGjeNb, c = e / kGjeNb;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int q = 0; q < kGjeNb; ++q) {
      const double2 a = m1[r][q], b = y1[q][c];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
    zr[r][c] = sr;
    zi[r][c] = si;
  }
  __syncthreads();
  // 3. Y(other rows) -= P Z on the matrix cores: 16-row blocks, two 16-column blocks
  const int nrb = (n + 15) / 16;
  for (int rb = wave; rb < nrb; rb += kUpdWaves) {
    const int r0 = rb * 16;  // the pivot rows have zero multipliers and are masked below
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      if (cb * 16 >= nc) break;
      dvec4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < kGjeNb; kk += 4) {
        // multipliers: the panel columns of W (rows below k: current values;
        // rows below the pivot block: their original values, already
        // interchanged by the panel kernel; pivot rows are masked below)
        const int row = r0 + (lane & 15), kq = kk + (lane >> 4);
        const double2 a = (row < n && kq < nb) ? gld(W + (size_t)(k + kq) * n + row) : make_double2(0.0, 0.0);
        const double br = zr[kq][cb * 16 + (lane & 15)], bi = zi[kq][cb * 16 + (lane & 15)];
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, br, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, bi, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bi, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, br, acci, 0, 0, 0);
      }
      const int c = cb * 16 + (lane & 15);
      if (c < nc) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = r0 + (lane >> 4) + 4 * q;
          if (row < n && !(row >= k && row < k + nb)) {
            cplx* p = W + (size_t)(c0 + c) * n + row;
            double2 v = gld(p);
            v.x -= accr[q];
            v.y -= acci[q];
            gst(p, v);
          }
        }
      }
    }
  }
  // 4. pivot rows receive Z
  for (int e = tid; e < nb * nc; e += kUpdThreads) {
    const int r = e % nb, c = e / nb;
    gst(W + (size_t)(c0 + c) * n + k + r, make_double2(zr[r][c], zi[r][c]));
  }
}

// y = g - U1 x1 - U2 x2 for right-hand-side column blockIdx.z, one workgroup
// per 64 rows, four wavefronts split the columns of U1, U2
__global__ __launch_bounds__(256) void gemv_step_kernel(const GemvDesc* __restrict__ descs) {
  const GemvDesc& D = descs[blockIdx.y];
  const int rc = blockIdx.z;
  if (rc >= D.r) return;
  const int row = blockIdx.x * 64 + (threadIdx.x & 63);
  const int wave = threadIdx.x >> 6;
  const cplx* x1 = D.x1 + (size_t)rc * D.m1;
  const cplx* x2 = D.x2 + (size_t)rc * D.m2;
  __shared__ double2 part[4][64];
  double2 acc = make_double2(0.0, 0.0);
  if (row < D.n) {
    for (int j = wave; j < D.m1; j += 4) {
      const double2 u = gld(D.U1 + (size_t)j * D.n + row), x = gld(x1 + j);
      acc.x += u.x * x.x - u.y * x.y;
      acc.y += u.x * x.y + u.y * x.x;
    }
    for (int j = wave; j < D.m2; j += 4) {
      const double2 u = gld(D.U2 + (size_t)j * D.n + row), x = gld(x2 + j);
      acc.x += u.x * x.x - u.y * x.y;
      acc.y += u.x * x.y + u.y * x.x;
    }
  }
  part[wave][threadIdx.x & 63] = acc;
  __syncthreads();
  if (wave == 0 && row < D.n) {
    double2 s = gld(D.g + (size_t)rc * D.n + row);
    for (int w = 0; w < 4; ++w) {
      s.x -= part[w][threadIdx.x].x;
      s.y -= part[w][threadIdx.x].y;
    }
    gst(D.y + (size_t)rc * D.n + row, s);
  }
}

// Right-hand-side kernel: 8 wavefronts, wave w owns the 16-row blocks
// w, w + 8, ... of the LDS tile.  Per step each wave loads the multipliers of
// its blocks and M1 into registers first (their latency overlaps the row
// interchanges), forms Z = M1 Y(pivot rows) itself on the matrix cores (the
// accumulator layout of Z is exactly the B-operand layout of the update
// product), then updates its blocks in LDS.
constexpr int kRhsWaves = 8;

// TC right-hand-side columns per workgroup (16, or 8 for orders up to
// kGjeMaxN, whose 16-column tile would not fit in LDS: then lanes of columns
// 8..15 carry zeros through the 16-wide matrix-core products)
// Steps [s0, s1) are replayed (clipped to each matrix's step count); the
// grid may be smaller than the number of tiles, workgroups then loop over
// tiles, so that a launch can run beside the panel chain on part of the chip.
template <int TC, int MAXN>
__global__ __launch_bounds__(kRhsWaves * 64) void gje_rhs_kernel(const GjeDesc* __restrict__ descs, int nbatch,
                                                                 int tiles_per, int s0, int s1) {
  constexpr int NBLK = (MAXN / 16 + kRhsWaves - 1) / kRhsWaves;  // row blocks per wave
  constexpr int PF = NBLK <= 5 ? NBLK : 4;  // blocks whose multipliers are prefetched (register budget)
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  const bool cl = lr < TC;
  __shared__ double2 Y[MAXN][TC];
  for (int tile = blockIdx.x; tile < nbatch * tiles_per; tile += gridDim.x) {
  const GjeDesc& D = descs[tile / tiles_per];
  const int n = D.n;
  const int c0 = n + (tile % tiles_per) * TC;
  if (c0 >= D.ncol) continue;
  const int nc = min(TC, D.ncol - c0);
  cplx* W = D.W;
  for (int e = tid; e < n * TC; e += kRhsWaves * 64) {
    const int r = e % n, c = e / n;
    Y[r][c] = c < nc ? gld(W + (size_t)(c0 + c) * n + r) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int nsteps = min(s1, (n + kGjeNb - 1) / kGjeNb);
  for (int sidx = s0; sidx < nsteps; ++sidx) {
    const int k = sidx * kGjeNb;
    const int nb = min(kGjeNb, n - k);
    const int* piv = D.piv + (size_t)sidx * kGjePivStride;
    const cplx* M1 = D.M1 + (size_t)sidx * kGjeNb * kGjeNb;
    // 0. operands of this step into registers: multipliers of my row blocks
    //    (lane: row r0 + lr, column kk + lq) and M1 (lane: row lr, column kk + lq)
    double2 pa[PF][4], ma[4];
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int row = (wave + j * kRhsWaves) * 16 + lr;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int kq = 4 * kk + lq;
        pa[j][kk] = (row < n && kq < nb) ? gld(W + (size_t)(k + kq) * n + row) : make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) ma[kk] = gld(M1 + (size_t)(4 * kk + lq) * kGjeNb + lr);
    // 1. this step's row interchanges (at most 2 NB pairs x TC columns)
    const int naff = piv[0];
    const int e0 = tid;
    const int cA = e0 % TC;
    const int dA = e0 < naff * TC ? piv[1 + e0 / TC] : -1;
    double2 vA = make_double2(0.0, 0.0);
    if (dA >= 0) vA = Y[piv[1 + 2 * kGjeNb + e0 / TC]][cA];
    __syncthreads();
    if (dA >= 0) Y[dA][cA] = vA;
    __syncthreads();
    // 2. Z = M1 Y(pivot rows), rows of Y beyond nb read as zero
    dvec4 zr = {0, 0, 0, 0}, zi = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int q = 4 * kk + lq;
      const double2 b = (q < nb && cl) ? Y[k + q][lr] : make_double2(0.0, 0.0);
      const double2 a = ma[kk];
      zr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, zr, 0, 0, 0);
      zr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, zr, 0, 0, 0);
      zi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, zi, 0, 0, 0);
      zi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, zi, 0, 0, 0);
    }
    __syncthreads();  // every wave has read the pivot rows
    // 3. Y(other rows) -= P Z; the pivot block (k is a multiple of 16, and
    //    nb < 16 only in the last block) receives Z.  Register q of Z holds
    //    row 4 q + lq, column lr: the B operand of step kk = q.
#pragma unroll
    for (int j = 0; j < NBLK; ++j) {
      const int r0 = (wave + j * kRhsWaves) * 16;
      if (r0 >= n) break;
      if (r0 == k) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = lq + 4 * q;
          if (cl && r0 + rr < n) Y[r0 + rr][lr] = make_double2(zr[q], zi[q]);
        }
        continue;
      }
      double2 pb[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int row = r0 + lr, kq = 4 * kk + lq;
        if (j < PF)
          pb[kk] = pa[j < PF ? j : 0][kk];
        else
          pb[kk] = (row < n && kq < nb) ? gld(W + (size_t)(k + kq) * n + row) : make_double2(0.0, 0.0);
      }
      dvec4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double2 a = pb[kk];
        const double br = zr[kk], bi = zi[kk];
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, br, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, bi, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bi, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, br, acci, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = r0 + lq + 4 * q;
        if (cl && row < n) {
          double2 y = Y[row][lr];
          y.x -= accr[q];
          y.y -= acci[q];
          Y[row][lr] = y;
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < n * TC; e += kRhsWaves * 64) {
    const int r = e % n, c = e / n;
    if (c < nc) gst(W + (size_t)(c0 + c) * n + r, Y[r][c]);
  }
  __syncthreads();  // before the next tile refills the LDS tile
  }
}

void gje_init() {}

void launch_gje_panel(const GjeDesc* d, int nbatch, int k, int max_n, hipStream_t st) {
  const size_t lds = (size_t)(max_n - k) * kGjeNb * sizeof(double2);
  (void)lds;
  if (nbatch > 0 && max_n > k) hipLaunchKernelGGL(gje_panel_kernel, dim3(nbatch), dim3(kPanelThreads), 0, st, d, k);
}
void launch_gje_update(const GjeDesc* d, int nbatch, int k, int max_n, int lo, int hi, hipStream_t st) {
  const int width = std::min(max_n - k - kGjeNb, hi) - lo;
  if (nbatch > 0 && width > 0) {
    const int tiles = (width - 1) / kGjeCols + 1;
    hipLaunchKernelGGL(gje_update_kernel, dim3(tiles, nbatch), dim3(kUpdThreads), 0, st, d, k, lo, hi);
  }
}
void launch_gje_rhs(const GjeDesc* d, int nbatch, int max_rhs, int max_n, int s0, int s1, int max_blocks,
                    hipStream_t st) {
  if (nbatch <= 0 || max_rhs <= 0 || s1 <= s0) return;
  const bool wide = max_n <= kRhsMaxN16;
  const int tiles_per = wide ? (max_rhs + 15) / 16 : (max_rhs + 7) / 8;
  const int total = nbatch * tiles_per;
  const int grid = max_blocks > 0 ? std::min(total, max_blocks) : total;
  if (wide)
    hipLaunchKernelGGL((gje_rhs_kernel<16, kRhsMaxN16>), dim3(grid), dim3(kRhsWaves * 64), 0, st, d, nbatch,
                       tiles_per, s0, s1);
  else
    hipLaunchKernelGGL((gje_rhs_kernel<8, kGjeMaxN>), dim3(grid), dim3(kRhsWaves * 64), 0, st, d, nbatch, tiles_per,
                       s0, s1);
}
void launch_gemv_step(const GemvDesc* d, int nbatch, int max_n, int max_r, hipStream_t st) {
  if (nbatch > 0 && max_n > 0 && max_r > 0)
    hipLaunchKernelGGL(gemv_step_kernel, dim3((max_n + 63) / 64, nbatch, max_r), dim3(256), 0, st, d);
}

}  // namespace mlh

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
//   gje_update_kernel  one workgroup of 12 wavefronts per 16 trailing
//                      columns (32 columns and 8 wavefronts above order
//                      576): applies the row swaps, Z = M1 Y(pivot rows),
//                      Y(other rows) -= P Z on the FP64 matrix cores,
//                      Y(pivot rows) = Z; on levels with few matrices the
//                      trailing columns run on through the right-hand sides;
//   gje_step_kernel    panel k and the update of step k - NB in one launch
//                      (disjoint columns);
//   gje_premul_kernel  after the last step: P' = P M1 for every step, in
//                      place;
//   gje_rhs_kernel     then one workgroup per 16 (8 for n > 608) right-hand-
//                      side columns keeps its tile in LDS and applies every
//                      step's interchanges and Y -= P' Y(pivot rows) to it.
//                      The right-hand sides thus cross HBM once instead of
//                      once per step;
//   gemv_step_kernel   back substitution of the cyclic reduction,
//                      y = g - U1 x1 - U2 x2.
#include <algorithm>

#include "internal.hpp"

namespace mlh {

typedef double dvec4 __attribute__((ext_vector_type(4)));

__device__ inline double2 gld(const cplx* p) { return ldc(p); }
__device__ inline void gst(cplx* p, double2 v) { stc(p, v.x, v.y); }
__device__ inline double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cinv2(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

// Panel kernel.  Thread t of the workgroup owns rows k + t + s NT (s < SLOTS)
// of the 16 panel columns, in registers.  It runs in three parts.
//  1. (k > 0) The previous step's transformation on these columns, rows >= k:
//     the old values, the previous interchanges and M1 arrive in one round of
//     loads and the pivot rows Y1 (and the rows the interchanges bring in) in
//     a second; Z = M1 Y1 goes to LDS; Y -= P Z runs on the matrix cores 16
//     rows at a time, each result block handed to the rows' owners through a
//     per-wave LDS tile.  The values reached are this step's start values;
//     they go back to W, where the update kernels read their multipliers.
//  2. LU with partial pivoting of rows k..n-1.  Rows are not moved: a row
//     that wins the pivot search for column c is marked and its values are
//     staged in LDS, so each column costs one workgroup barrier.  Every wave
//     reduces its candidates to one 32-bit key (|a|^2 to 2^-10, then the
//     complemented row offset, so that ties go to the lowest row) with DPP
//     moves; the candidate lanes form the reciprocal of their pivot while the
//     reduction runs, and the winning lane stages it with its row.
//  3. The tail, split over waves: wave 0 composes this step's interchanges
//     with ballots and applies them to the panel columns of W; wave 1 forms
//     M1 = (L11 U11)^-1; the other waves apply the previous step to the rows
//     above k (Z on its pivot rows, V - P Z above them).
constexpr int kPanelMaxWaves = 12;


// value of lane S of each group of four lanes (DPP quad permutation)
__device__ inline double quad_bcast(double v, int S) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(uint32_t)b, hi = (int)(uint32_t)(b >> 32);
  switch (S) {
    case 0:
      lo = __builtin_amdgcn_mov_dpp(lo, 0x00, 0xf, 0xf, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0x00, 0xf, 0xf, false);
      break;
    case 1:
      lo = __builtin_amdgcn_mov_dpp(lo, 0x55, 0xf, 0xf, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0x55, 0xf, 0xf, false);
      break;
    case 2:
      lo = __builtin_amdgcn_mov_dpp(lo, 0xaa, 0xf, 0xf, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0xaa, 0xf, 0xf, false);
      break;
    default:
      lo = __builtin_amdgcn_mov_dpp(lo, 0xff, 0xf, 0xf, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0xff, 0xf, 0xf, false);
      break;
  }
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// orders LDS traffic between the lanes of one wavefront
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// rows of one thread and the LU state shared by the per-column steps
template <int SLOTS>
struct PanelRows {
  double2 a[SLOTS][kGjeNb];
  int pidx[SLOTS];  // pivot order of the row, -1 while still eligible, kGjeNb for no row
  int singular;
};

struct PanelShared {  // per-column exchange, double-buffered over columns
  uint32_t key[2][kPanelMaxWaves];
  double2 row[2][kPanelMaxWaves][kGjeNb];
  double2 ip[2][kPanelMaxWaves];
  int spiv[kGjeNb];       // global row of each pivot
  double2 ipiv[kGjeNb];   // reciprocal of each pivot
};

// maximum of x over the wavefront, returned in every lane
__device__ inline uint32_t wave_max_u32(uint32_t x) {
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true));  // row_shr:1
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true));  // row_shr:2
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true));  // row_shr:4
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true));  // row_shr:8
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, true));  // row_bcast:15
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, true));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// 1/v for the pivot: hardware reciprocal of |v|^2 refined by two Newton
// steps (zero for v = 0; an exactly singular column is reported anyway)
__device__ inline double2 pivot_recip(double vx, double vy) {
  const double d = vx * vx + vy * vy;
  double r = __builtin_amdgcn_rcp(d);
  r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
  r = d != 0.0 ? r : 0.0;
  return make_double2(vx * r, -vy * r);
}

// Pivot key of a candidate row: the high word of |a|^2 without its ten
// lowest bits, plus one (zero means no eligible row), over ten bits of
// complemented row offset.  Keys are unique, the largest is the pivot, and
// the pivot is within 2^-10 of the largest |a|^2 of the column (ties to the
// lowest row), which keeps partial pivoting's growth bound.
constexpr int kKeyRowBits = 10;
__device__ inline uint32_t pivot_key32(double vx, double vy, int rel) {
  const double m2 = vx * vx + vy * vy;
  const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(m2) >> 32);
  return (((hi >> kKeyRowBits) + 1u) << kKeyRowBits) | (uint32_t)((1 << kKeyRowBits) - 1 - rel);
}

// one column of the panel LU; C is a template parameter so that every
// register index is static.  Waves without rows (all past n) only keep the
// barriers; their keys stay zero.
template <int NT, int SLOTS, int C>
__device__ __forceinline__ void panel_column(PanelRows<SLOTS>& st, PanelShared& sh, int nb, int k, int tid,
                                             bool active) {
  if (C >= nb) return;
  constexpr int NW = NT / 64;
  const int lane = tid & 63, wave = tid >> 6;
  const int buf = C & 1;
  if (active) {
    uint32_t key = 0;
    double cx = 0.0, cy = 0.0;  // scalar selects keep the rows in registers
    int csl = 0;
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) {
      const double vx = st.a[sl][C].x, vy = st.a[sl][C].y;
      const uint32_t kk = st.pidx[sl] < 0 ? pivot_key32(vx, vy, tid + sl * NT) : 0u;
      const bool better = kk > key;
      key = better ? kk : key;
      csl = better ? sl : csl;
      cx = better ? vx : cx;
      cy = better ? vy : cy;
    }
    const double2 cip = pivot_recip(cx, cy);
    const uint32_t wmax = wave_max_u32(key);
    const int wrel = (1 << kKeyRowBits) - 1 - (int)(wmax & ((1u << kKeyRowBits) - 1));
    const int wl = (SLOTS == 1 ? wrel : wrel % NT) & 63;  // lane holding the wave's candidate
    // cross-lane reads stay in uniform control flow
    const double2 wip = make_double2(readlane_d(cip.x, wl), readlane_d(cip.y, wl));
    if (lane == 0) {
      sh.key[buf][wave] = wmax;
      sh.ip[buf][wave] = wip;
    }
    if (wmax != 0 && key == wmax) {  // the later columns of the candidate row
      const bool s0 = SLOTS == 1 || csl == 0;
#pragma unroll
      for (int j = C + 1; j < kGjeNb; ++j) {
        const double rx = s0 ? st.a[0][j].x : st.a[SLOTS - 1][j].x;
        const double ry = s0 ? st.a[0][j].y : st.a[SLOTS - 1][j].y;
        sh.row[buf][wave][j] = make_double2(rx, ry);
      }
    }
  }
  __syncthreads();
  if (!active) return;
  uint32_t kv[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) kv[w] = sh.key[buf][w];
#pragma unroll
  for (int s = 1; s < NW; s *= 2)
#pragma unroll
    for (int w = 0; w + s < NW; w += 2 * s) kv[w] = max(kv[w], kv[w + s]);
  const uint32_t kb = kv[0];
  const int rel = (1 << kKeyRowBits) - 1 - (int)(kb & ((1u << kKeyRowBits) - 1));  // pivot row - k
  const int wb = (SLOTS == 1 ? rel : rel % NT) >> 6;                                  // the wave that staged it
  if ((kb >> kKeyRowBits) <= 1u && st.singular == 0) st.singular = k + C + 1;
  const double2 ip = sh.ip[buf][wb];
  double2 prow[kGjeNb];
#pragma unroll
  for (int j = C + 1; j < kGjeNb; ++j) prow[j] = sh.row[buf][wb][j];
  if (tid == 0) {
    sh.spiv[C] = k + rel;
    sh.ipiv[C] = ip;
  }
#pragma unroll
  for (int sl = 0; sl < SLOTS; ++sl) {
    if (tid + sl * NT == rel) {
      st.pidx[sl] = C;
    } else if (st.pidx[sl] < 0) {
      const double2 v = st.a[sl][C];
      const double2 l = make_double2(v.x * ip.x - v.y * ip.y, v.x * ip.y + v.y * ip.x);
      st.a[sl][C] = l;
#pragma unroll
      for (int j = C + 1; j < kGjeNb; ++j) {
        double2 y = st.a[sl][j];
        y.x = __builtin_fma(-l.x, prow[j].x, __builtin_fma(l.y, prow[j].y, y.x));
        y.y = __builtin_fma(-l.x, prow[j].y, __builtin_fma(-l.y, prow[j].x, y.y));
        st.a[sl][j] = y;
      }
    }
  }
}

template <int NT, int SLOTS, int C>
struct PanelColumns {
  static __device__ __forceinline__ void run(PanelRows<SLOTS>& st, PanelShared& sh, int nb, int k, int tid,
                                             bool active) {
    panel_column<NT, SLOTS, C>(st, sh, nb, k, tid, active);
    PanelColumns<NT, SLOTS, C + 1>::run(st, sh, nb, k, tid, active);
  }
};
template <int NT, int SLOTS>
struct PanelColumns<NT, SLOTS, kGjeNb> {
  static __device__ __forceinline__ void run(PanelRows<SLOTS>&, PanelShared&, int, int, int, bool) {}
};

template <int NT, int SLOTS>
__device__ __forceinline__ void panel_body(const GjeDesc* __restrict__ descs, int k, int b) {
  static_assert(NT % 64 == 0 && NT / 64 <= kPanelMaxWaves && NT >= 256, "panel workgroup shape");
  constexpr int NW = NT / 64;
  const GjeDesc& D = descs[b];
  const int n = D.n;
  if (k >= n) return;
  const int nb = min(kGjeNb, n - k);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  cplx* W = D.W;
  __shared__ PanelShared sh;
  __shared__ int sdst[2 * kGjeNb], ssrc[2 * kGjeNb], snaff;
  __shared__ double2 m1[kGjeNb][kGjeNb + 1];
  __shared__ double2 ys[kGjeNb][kGjeNb];
  __shared__ double2 zs[kGjeNb][kGjeNb];
  __shared__ double2 tile[NW][kGjeNb][kGjeNb + 1];
  __shared__ double2 lu11[kGjeNb][kGjeNb + 1];
  __shared__ int pdst[2 * kGjeNb], psrc[2 * kGjeNb], below[kGjeNb];

  PanelRows<SLOTS> st;
  st.singular = 0;
#pragma unroll
  for (int sl = 0; sl < SLOTS; ++sl) {
    const int r = k + tid + sl * NT;
    st.pidx[sl] = r < n ? -1 : kGjeNb;
#pragma unroll
    for (int j = 0; j < kGjeNb; ++j)
      st.a[sl][j] = (r < n && j < nb) ? gld(W + (size_t)(k + j) * n + r) : make_double2(0.0, 0.0);
  }
  const int kp = k - kGjeNb;
  if (k > 0) {
    // first load round: the previous step's interchanges and M1 (the old values of
    // our rows are in flight above)
    const auto pivp = gmem(D.piv + (size_t)(kp / kGjeNb) * kGjePivStride);
    const cplx* M1p = D.M1 + (size_t)(kp / kGjeNb) * kGjeNb * kGjeNb;
    if (tid == 0) snaff = pivp[0];
    if (tid < 2 * kGjeNb) {
      sdst[tid] = pivp[1 + tid];
      ssrc[tid] = pivp[1 + 2 * kGjeNb + tid];
    }
    if (tid < kGjeNb * kGjeNb) m1[tid % kGjeNb][tid / kGjeNb] = gld(M1p + tid);  // column-major M1
    // the multipliers of the previous step for our row blocks (MFMA A
    // operand: lane (lq, lr) holds P[r0 + lr][4 kk + lq])
    // (first slot only: registers)
    double2 pa[4][4];
    {
      constexpr int sl = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int row = k + sl * NT + wave * 64 + i * 16 + lr;
          pa[i][kk] = row < n ? gld(W + (size_t)(kp + 4 * kk + lq) * n + row) : make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    // second load round: Y1 = the previous pivot rows after the interchanges, and the
    // rows the interchanges bring into our rows (all from rows kp..k-1)
    const int naff = snaff;
    if (tid < kGjeNb * kGjeNb) {
      const int i = tid % kGjeNb, c = tid / kGjeNb;
      int src = kp + i;
      for (int t = 0; t < naff; ++t)
        if (sdst[t] == kp + i) src = ssrc[t];
      ys[i][c] = c < nb ? gld(W + (size_t)(k + c) * n + src) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) {
      const int r = k + tid + sl * NT;
      int src = -1;
      for (int t = 0; t < naff; ++t)
        if (sdst[t] == r) src = ssrc[t];
      if (src >= 0)
#pragma unroll
        for (int j = 0; j < kGjeNb; ++j)
          st.a[sl][j] = j < nb ? gld(W + (size_t)(k + j) * n + src) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (tid < kGjeNb * kGjeNb) {  // Z = M1 Y1
      const int i = tid % kGjeNb, c = tid / kGjeNb;
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < kGjeNb; ++q) {
        const double2 x = m1[i][q], y = ys[q][c];
        sr += x.x * y.x - x.y * y.y;
        si += x.x * y.y + x.y * y.x;
      }
      zs[i][c] = make_double2(sr, si);
    }
    __syncthreads();
    // Y -= P Z for our rows, 16 at a time: lane (lq, lr) holds P[r0 + lr][4 kk + lq]
    // and receives (P Z)[r0 + lq + 4 q][lr]
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r0 = k + sl * NT + wave * 64 + i * 16;
        if (r0 >= n) break;
        // three real products per complex one: re = K1 - K3, im = K1 + K2
        // with K1 = (Ar + Ai) Br, K2 = Ar (Bi - Br), K3 = Ai (Br + Bi); K2
        // goes on top of K1 in a second pass, so that two accumulators suffice
        double2 a[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int row = r0 + lr;
          a[kk] = sl == 0 ? pa[i][kk]
                          : (row < n ? gld(W + (size_t)(kp + 4 * kk + lq) * n + row) : make_double2(0.0, 0.0));
        }
        dvec4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double2 b = zs[4 * kk + lq][lr];
          acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk].x + a[kk].y, b.x, acci, 0, 0, 0);
          accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[kk].y, b.x + b.y, accr, 0, 0, 0);
        }
        accr += acci;
        asm volatile("" ::: "memory");  // Z is read again below rather than held in registers
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double2 b = zs[4 * kk + lq][lr];
          acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk].x, b.y - b.x, acci, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) tile[wave][lq + 4 * q][lr] = make_double2(accr[q], acci[q]);
        wave_lds_sync();
        if (lq == i) {
#pragma unroll
          for (int j = 0; j < kGjeNb; ++j) {
            const double2 t = tile[wave][lr][j];
            st.a[sl][j].x -= t.x;
            st.a[sl][j].y -= t.y;
          }
        }
        wave_lds_sync();
      }
    }
    // this step's start values back to W (their loads settled first, so
    // that the stores issue back to back)
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
#pragma unroll
    for (int sl = 0; sl < SLOTS; ++sl) {
      const int r = k + tid + sl * NT;
      if (r < n)
#pragma unroll
        for (int j = 0; j < kGjeNb; ++j)
          if (j < nb) gst(W + (size_t)(k + j) * n + r, st.a[sl][j]);
    }
  } else {
    // the rows just loaded: wait here, so that the join below does not also
    // wait for the start-value stores of the k > 0 path
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
  }
  // waves whose rows all lie past n sit out the column steps (their keys are zero)
  const bool active = k + (tid & ~63) < n;
  if (tid < 2 * kPanelMaxWaves) sh.key[tid / kPanelMaxWaves][tid % kPanelMaxWaves] = 0u;
  __syncthreads();
  PanelColumns<NT, SLOTS, 0>::run(st, sh, nb, k, tid, active);
  if (tid == 0 && st.singular != 0) atomicCAS(D.info, 0, st.singular);
  // the factored pivot block: row of pivot c holds L11 (j < c) and U11 (j >= c)
#pragma unroll
  for (int sl = 0; sl < SLOTS; ++sl)
    if (st.pidx[sl] >= 0 && st.pidx[sl] < kGjeNb)
#pragma unroll
      for (int j = 0; j < kGjeNb; ++j) lu11[st.pidx[sl]][j] = st.a[sl][j];
  if (tid >= nb && tid < kGjeNb) {
#pragma unroll
    for (int j = 0; j < kGjeNb; ++j) lu11[tid][j] = make_double2(0.0, 0.0);
    sh.ipiv[tid] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (wave == 0) {
    // this step's row permutation as (destination, source) pairs of global
    // rows: pivot q (row spiv[q], never moved in registers) goes to k + q;
    // rows of positions k..k+nb-1 that were not chosen fill, in order, the
    // rows that the pivots from below the block vacated, in pivot order.
    // piv[0] = count, piv[1..] destinations, piv[1+2NB..] sources,
    // piv[1+4NB+q] the row of pivot q.
    const int q = lane;
    const int p = q < nb ? sh.spiv[q] : -1;
    bool chosen = false;
    for (int t = 0; t < nb; ++t) chosen |= (sh.spiv[t] == k + q);
    const bool isA = q < nb && p != k + q;
    const bool isB = q < nb && p >= k + nb;
    const bool isU = q < nb && !chosen;
    const uint64_t bA = __ballot(isA), bB = __ballot(isB), bU = __ballot(isU);
    const uint64_t lt = (1ull << lane) - 1ull;
    const int nA = __popcll(bA);
    if (isB) below[__popcll(bB & lt)] = p;
    wave_lds_sync();
    const auto piv = gmem(D.piv + (size_t)(k / kGjeNb) * kGjePivStride);
    if (isA) {
      const int t = __popcll(bA & lt);
      pdst[t] = k + q;
      psrc[t] = p;
      piv[1 + t] = k + q;
      piv[1 + 2 * kGjeNb + t] = p;
    }
    if (isU) {
      const int u = __popcll(bU & lt), t = nA + u;
      pdst[t] = below[u];
      psrc[t] = k + q;
      piv[1 + t] = below[u];
      piv[1 + 2 * kGjeNb + t] = k + q;
    }
    const int na = nA + __popcll(bU);
    if (lane == 0) piv[0] = na;
    if (q < nb) piv[1 + 4 * kGjeNb + q] = p;  // the row holding pivot q before the interchanges
    wave_lds_sync();
    // apply it to the panel columns of W (this step's start values): every
    // source is read before any destination is written
    double2 v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = lane + 64 * m;
      v[m] = e < na * nb ? gld(W + (size_t)(k + e / na) * n + psrc[e % na]) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = lane + 64 * m;
      if (e < na * nb) gst(W + (size_t)(k + e / na) * n + pdst[e % na], v[m]);
    }
  } else if (wave == 1) {
    // M1 = (L11 U11)^{-1}: lane 4 c + g holds rows g + 4 q of column c;
    // X = L11^{-1} by row operations, then M1 = U11^{-1} X with the pivot
    // reciprocals of the factorisation
    const int c = lane >> 2, g = lane & 3;
    double2 x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = make_double2(g + 4 * q == c ? 1.0 : 0.0, 0.0);
    // branch-free: each lane reads its four entries of the pivot column and
    // keeps the updates of its rows that step r touches; rows that no lane
    // of a quad can touch at step r are skipped at compile time
#pragma unroll
    for (int r = 0; r < kGjeNb - 1; ++r) {
      const double2 xr = make_double2(quad_bcast(x[r / 4].x, r % 4), quad_bcast(x[r / 4].y, r % 4));
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (4 * q + 3 <= r) continue;
        const int i = g + 4 * q;
        const double2 l = lu11[i][r];
        const double tx = __builtin_fma(-l.x, xr.x, __builtin_fma(l.y, xr.y, x[q].x));
        const double ty = __builtin_fma(-l.x, xr.y, __builtin_fma(-l.y, xr.x, x[q].y));
        x[q].x = i > r ? tx : x[q].x;
        x[q].y = i > r ? ty : x[q].y;
      }
    }
#pragma unroll
    for (int r = kGjeNb - 1; r >= 0; --r) {
      const double2 y = make_double2(quad_bcast(x[r / 4].x, r % 4), quad_bcast(x[r / 4].y, r % 4));
      const double2 d = sh.ipiv[r];
      const double2 xr = make_double2(y.x * d.x - y.y * d.y, y.x * d.y + y.y * d.x);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (4 * q > r) continue;
        const int i = g + 4 * q;
        const double2 u = lu11[i][r];
        const double tx = __builtin_fma(-u.x, xr.x, __builtin_fma(u.y, xr.y, x[q].x));
        const double ty = __builtin_fma(-u.x, xr.y, __builtin_fma(-u.y, xr.x, x[q].y));
        x[q].x = i == r ? xr.x : (i < r ? tx : x[q].x);
        x[q].y = i == r ? xr.y : (i < r ? ty : x[q].y);
      }
    }
    cplx* M1 = D.M1 + (size_t)(k / kGjeNb) * kGjeNb * kGjeNb;
#pragma unroll
    for (int q = 0; q < 4; ++q) gst(M1 + (size_t)c * kGjeNb + g + 4 * q, c < nb ? x[q] : make_double2(0.0, 0.0));
  } else if (k > 0) {
    // the previous step on rows above k: its pivot rows kp..k-1 receive Z,
    // rows above them V - P Z (old values as the accumulators)
    const int wt = tid - 128;
    for (int e = wt; e < kGjeNb * kGjeNb; e += NT - 128) {
      const int i = e % kGjeNb, c = e / kGjeNb;
      if (c < nb) gst(W + (size_t)(k + c) * n + kp + i, zs[i][c]);
    }
    constexpr int G = 3;  // row blocks in flight per wave
    const int nrb = kp / 16;
    for (int b0 = wave - 2; b0 < nrb; b0 += G * (NW - 2)) {
      double2 pa[G][4];
      dvec4 vr[G], vi[G];
#pragma unroll
      for (int h = 0; h < G; ++h) {
        const int rb = b0 + h * (NW - 2);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          pa[h][kk] = ldc_sel(W + (size_t)(kp + 4 * kk + lq) * n + min(rb, nrb - 1) * 16 + lr, rb < nrb);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double2 v =
              ldc_sel(W + (size_t)(k + min(lr, nb - 1)) * n + min(rb, nrb - 1) * 16 + lq + 4 * q, rb < nrb && lr < nb);
          vr[h][q] = v.x;
          vi[h][q] = v.y;
        }
      }
#pragma unroll
      for (int h = 0; h < G; ++h) {
        const int rb = b0 + h * (NW - 2);
        if (rb >= nrb) break;
        // V - P Z in three real products: V.r - K1 + K3, V.i - K1 - K2
        dvec4 k1 = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double2 a = pa[h][kk], b = zs[4 * kk + lq][lr];
          k1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x, k1, 0, 0, 0);
          vi[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.x, b.y - b.x, vi[h], 0, 0, 0);
          vr[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x + b.y, vr[h], 0, 0, 0);
        }
        vr[h] -= k1;
        vi[h] -= k1;
        if (lr < nb)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            gst(W + (size_t)(k + lr) * n + rb * 16 + lq + 4 * q, make_double2(vr[h][q], vi[h][q]));
      }
    }
  }
}

template <int NT, int SLOTS>
__global__ __launch_bounds__(NT) void gje_panel_kernel(const GjeDesc* __restrict__ descs, int k) {
  panel_body<NT, SLOTS>(descs, k, blockIdx.x);
}

// Update kernel: one workgroup of 12 waves per 16 columns of the diagonal
// block, columns [k + nb + lo, min(n, k + nb + hi)), every row (orders up to
// kUpdMaxN); the right-hand-side columns are left to gje_rhs_kernel, after
// all steps.  Each wave owns up to kUpdRbw 16-row blocks.  Latency decides
// this kernel at the deep levels of the reduction, so its global traffic
// comes in two dependent rounds: (1) the interchanges, M1, the multipliers P
// and the old values of its rows, all at once; (2) the rows the interchanges
// move and the pivot rows Y1.  An interchanged row then takes its new value
// from LDS instead of being scattered through memory first.  The workgroup
// spans all rows because every row of its columns needs the old values of
// the interchanged and pivot rows.
constexpr int kUpdWaves = 12;
constexpr int kUpdRbw = 3;
constexpr int kUpdMaxN = kUpdWaves * kUpdRbw * 16;  // 576
constexpr int kUpdCols = 16;
constexpr int kUpdWideThreads = 512;
constexpr int kUpdWideWaves = kUpdWideThreads / 64;
constexpr int kUpdWideCols = 32;

// Step k on the columns from min(k + nb + lo, n) on: up to k + nb + hi
// within the diagonal block, or with rhs through the right-hand-side
// columns as well (Gauss-Jordan on [D | B] leaves D^{-1} B in place of B).
// The columns [k + nb, k + nb + lo) of the block are the next panel's.
__device__ __forceinline__ void update_body(const GjeDesc* __restrict__ descs, int k, int lo, int hi, int tx,
                                            int b, bool rhs) {
  const GjeDesc& D = descs[b];
  const int n = D.n;
  if (k >= n) return;
  const int nb = min(kGjeNb, n - k);
  const int cend = min(rhs ? D.ncol : n, k + nb + hi);
  const int c0 = min(k + nb + lo, n) + tx * kUpdCols;
  if (c0 >= cend) return;
  const int nc = min(kUpdCols, cend - c0);
  const auto piv = gmem(D.piv + (size_t)(k / kGjeNb) * kGjePivStride);
  const cplx* M1 = D.M1 + (size_t)(k / kGjeNb) * kGjeNb * kGjeNb;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  cplx* W = D.W;
  __shared__ int sdst[2 * kGjeNb], ssrc[2 * kGjeNb], snaff;
  __shared__ short rowmap[kUpdMaxN];  // stage slot of a row an interchange overwrites, else -1
  __shared__ double2 m1[kGjeNb][kGjeNb + 1];
  __shared__ double2 stage[2 * kGjeNb][kUpdCols];
  __shared__ double2 y1[kGjeNb][kUpdCols];
  __shared__ double2 zs[kGjeNb][kUpdCols];
  // first load round
  if (tid == 0) snaff = piv[0];
  if (tid < 2 * kGjeNb) {
    sdst[tid] = piv[1 + tid];
    ssrc[tid] = piv[1 + 2 * kGjeNb + tid];
  }
  if (tid < kGjeNb * kGjeNb) m1[tid % kGjeNb][tid / kGjeNb] = gld(M1 + tid);  // column-major M1
  for (int i = tid; i < n; i += kUpdWaves * 64) rowmap[i] = -1;
  // the old values are held as the accumulators of Y - P Z: register q of
  // lane (lq, lr) is row r0 + lq + 4 q of column c0 + lr
  double2 P[kUpdRbw][4];
  dvec4 Vr[kUpdRbw], Vi[kUpdRbw];
#pragma unroll
  for (int j = 0; j < kUpdRbw; ++j) {
    const int r0 = (wave + kUpdWaves * j) * 16;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int row = r0 + lr, kq = 4 * kk + lq;
      // clamped, not masked: a row past n only feeds results that are not
      // stored, and a column past nb meets the zero rows of Z
      P[j][kk] = ldc(W + (uint32_t)((k + min(kq, nb - 1)) * n + min(row, n - 1)));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // real and imaginary parts straight into the accumulators
      const int row = r0 + lq + 4 * q;
      const auto vp = gmem(reinterpret_cast<const double*>(W + (uint32_t)((c0 + min(lr, nc - 1)) * n + min(row, n - 1))));
      Vr[j][q] = vp[0];
      Vi[j][q] = vp[1];
    }
  }
  __syncthreads();
  // second load round: the rows the interchanges move, and Y1 (the pivot rows after them)
  const int naff = snaff;
  if (tid < naff) rowmap[sdst[tid]] = (short)tid;
  for (int e = tid; e < naff * kUpdCols; e += kUpdWaves * 64) {
    const int t = e % naff, c = e / naff;
    stage[t][c] = c < nc ? gld(W + (size_t)(c0 + c) * n + ssrc[t]) : make_double2(0.0, 0.0);
  }
  if (tid < kGjeNb * kUpdCols) {
    const int r = tid % kGjeNb, c = tid / kGjeNb;
    int src = k + r;
    for (int t = 0; t < naff; ++t)
      if (sdst[t] == k + r) src = ssrc[t];
    y1[r][c] = (r < nb && c < nc) ? gld(W + (size_t)(c0 + c) * n + src) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (tid < kGjeNb * kUpdCols) {  // Z = M1 Y1
    const int r = tid % kGjeNb, c = tid / kGjeNb;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int q = 0; q < kGjeNb; ++q) {
      const double2 a = m1[r][q], b = y1[q][c];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
    }
    zs[r][c] = make_double2(sr, si);
  }
  __syncthreads();
  // Y(other rows) = Y(after the interchanges) - P Z on the matrix cores;
  // the pivot rows receive Z
#pragma unroll
  for (int j = 0; j < kUpdRbw; ++j) {
    const int r0 = (wave + kUpdWaves * j) * 16;
    if (r0 >= n) break;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = r0 + lq + 4 * q;
      const int m = row < n ? rowmap[row] : -1;
      if (m >= 0) {
        const double2 v = stage[m][lr];
        Vr[j][q] = v.x;
        Vi[j][q] = v.y;
      }
    }
    // three real products per complex one: V.r - K1 + K3, V.i - K1 - K2 with
    // K1 = (Pr + Pi) Zr, K2 = Pr (Zi - Zr), K3 = Pi (Zr + Zi)
    dvec4 k1 = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double2 a = P[j][kk], b = zs[4 * kk + lq][lr];
      k1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x, k1, 0, 0, 0);
      Vi[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.x, b.y - b.x, Vi[j], 0, 0, 0);
      Vr[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x + b.y, Vr[j], 0, 0, 0);
    }
    Vr[j] -= k1;
    Vi[j] -= k1;
    if (lr < nc) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = r0 + lq + 4 * q;
        if (row >= n) continue;
        const double2 v = (row >= k && row < k + nb) ? zs[row - k][lr] : make_double2(Vr[j][q], Vi[j][q]);
        gst(W + (size_t)(c0 + lr) * n + row, v);
      }
    }
  }
}

__global__ __launch_bounds__(kUpdWaves * 64) void gje_update_kernel(const GjeDesc* __restrict__ descs, int k, int lo,
                                                                    int hi, int rhs) {
  update_body(descs, k, lo, hi, blockIdx.x, blockIdx.y, rhs != 0);
}

// One launch per elimination step when every order is at most kUpdMaxN:
// workgroups [0, nbatch) factor panel k, the others apply step k - 16 to
// the columns from k + 16 on, one per (16 columns, matrix).  The two parts
// touch disjoint columns and depend only on earlier launches, so a level
// needs neither a second stream nor events, and the panel workgroups, which
// dispatch first, find their compute units free.
__global__ __launch_bounds__(kUpdWaves * 64) void gje_step_kernel(const GjeDesc* __restrict__ descs, int nbatch,
                                                                  int k, int utiles, int rhs) {
  if ((int)blockIdx.x < nbatch) {
    panel_body<kUpdWaves * 64, 1>(descs, k, blockIdx.x);
  } else {
    const int u = blockIdx.x - nbatch;
    update_body(descs, k - kGjeNb, kGjeNb, 1 << 30, u % utiles, u / utiles, rhs != 0);
  }
}

// Orders above kUpdMaxN: one workgroup of 16 waves per 32 columns, each wave
// walking its row blocks with the old values loaded as it goes.
__global__ __launch_bounds__(kUpdWideThreads) void gje_update_wide_kernel(const GjeDesc* __restrict__ descs, int k,
                                                                          int lo, int hi) {
  const GjeDesc& D = descs[blockIdx.y];
  const int n = D.n;
  if (k >= n) return;
  const int nb = min(kGjeNb, n - k);
  const int cend = min(n, k + nb + hi);
  const int c0 = k + nb + lo + blockIdx.x * kUpdWideCols;
  if (c0 >= cend) return;
  const int nc = min(kUpdWideCols, cend - c0);
  const auto piv = gmem(D.piv + (size_t)(k / kGjeNb) * kGjePivStride);
  const cplx* M1 = D.M1 + (size_t)(k / kGjeNb) * kGjeNb * kGjeNb;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  cplx* W = D.W;
  __shared__ double zr[kGjeNb][kUpdWideCols + 1], zi[kGjeNb][kUpdWideCols + 1];
  __shared__ double2 m1[kGjeNb][kGjeNb];
  __shared__ double2 y1[kGjeNb][kUpdWideCols];
  // 1. row interchanges of this step on our columns, as (destination, source)
  //    pairs composed by the panel kernel: stage the sources, then write back
  __shared__ int sdst[2 * kGjeNb], ssrc[2 * kGjeNb];
  __shared__ double2 stage[2 * kGjeNb][kUpdWideCols];
  const int naff = piv[0];
  if (tid < naff) {
    sdst[tid] = piv[1 + tid];
    ssrc[tid] = piv[1 + 2 * kGjeNb + tid];
  }
  for (int e = tid; e < kGjeNb * kGjeNb; e += kUpdWideThreads) m1[e % kGjeNb][e / kGjeNb] = gld(M1 + e);
  __syncthreads();
  for (int e = tid; e < naff * nc; e += kUpdWideThreads) {
    const int t = e % naff, c = e / naff;
    stage[t][c] = gld(W + (size_t)(c0 + c) * n + ssrc[t]);
  }
  __syncthreads();
  for (int e = tid; e < naff * nc; e += kUpdWideThreads) {
    const int t = e % naff, c = e / naff;
    gst(W + (size_t)(c0 + c) * n + sdst[t], stage[t][c]);
  }
  __syncthreads();
  // 2. Z = M1 Y1
  for (int e = tid; e < kGjeNb * kUpdWideCols; e += kUpdWideThreads) {
    const int r = e % kGjeNb, c = e / kGjeNb;
    y1[r][c] = (r < nb && c < nc) ? gld(W + (size_t)(c0 + c) * n + k + r) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int e = tid; e < kGjeNb * kUpdWideCols; e += kUpdWideThreads) {
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
  // 3. Y(other rows) -= P Z on the matrix cores: 16-row blocks times the
  //    16-column blocks of the tile; each row block's old values and
  //    multipliers are loaded in one round, before its products (8 % faster
  //    than loading the old values after the products).  The loads are
  //    clamped and unmasked, and every column block is multiplied, so that
  //    no select or branch makes the wave wait for a load before the last
  //    one is issued: rows past n and columns past nc are not stored, and
  //    multiplier columns past nb meet rows of Z that are zero (M1 is zero
  //    there)
  const int nrb = (n + 15) / 16;
#pragma unroll 1
  for (int rb = wave; rb < nrb; rb += kUpdWideWaves) {
    const int r0 = rb * 16;  // the pivot rows have zero multipliers and are masked below
    double2 a[kGjeNb / 4], v[kUpdWideCols / 16][4];
#pragma unroll
    for (int kk = 0; kk < kGjeNb; kk += 4) {
      // multipliers: the panel columns of W (rows below k: current values;
      // rows below the pivot block: their original values, already
      // interchanged by the panel kernel; pivot rows are masked below)
      const int row = min(r0 + (lane & 15), n - 1), kq = min(kk + (lane >> 4), nb - 1);
      a[kk / 4] = gld(W + (size_t)(k + kq) * n + row);
    }
#pragma unroll
    for (int cb = 0; cb < kUpdWideCols / 16; ++cb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = min(cb * 16 + (lane & 15), nc - 1), row = min(r0 + (lane >> 4) + 4 * q, n - 1);
        v[cb][q] = gld(W + (size_t)(c0 + c) * n + row);  // clamped: entries past nc or n are not stored
      }
    asm volatile("" ::: "memory");  // compiler barrier: the loads above are not sunk to their stores
#pragma unroll
    for (int cb = 0; cb < kUpdWideCols / 16; ++cb) {
      dvec4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < kGjeNb; kk += 4) {
        const int kq = kk + (lane >> 4);
        const double br = zr[kq][cb * 16 + (lane & 15)], bi = zi[kq][cb * 16 + (lane & 15)];
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk / 4].x, br, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[kk / 4].y, bi, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk / 4].x, bi, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk / 4].y, br, acci, 0, 0, 0);
      }
      const int c = cb * 16 + (lane & 15);
      if (c < nc) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = r0 + (lane >> 4) + 4 * q;
          if (row < n && !(row >= k && row < k + nb)) {
            double2 y = v[cb][q];
            y.x -= accr[q];
            y.y -= acci[q];
            gst(W + (size_t)(c0 + c) * n + row, y);
          }
        }
      }
    }
  }
  // 4. pivot rows receive Z
  for (int e = tid; e < nb * nc; e += kUpdWideThreads) {
    const int r = e % nb, c = e / nb;
    gst(W + (size_t)(c0 + c) * n + k + r, make_double2(zr[r][c], zi[r][c]));
  }
}

// y = g - U1 x1 - U2 x2 for right-hand-side column blockIdx.z, one workgroup
// per 64 rows; its sixteen wavefronts split the columns of U1, U2, each lane
// with four column loads in flight (clamped rows, no branch), and the
// partial sums meet in LDS
constexpr int kGemvWaves = 16;

__device__ __forceinline__ void gemv_cols(const cplx* U, const cplx* x, int m, int n, int row, int wave,
                                          double2& a0, double2& a1) {
  int j = wave;
  for (; j + 3 * kGemvWaves < m; j += 4 * kGemvWaves) {
    double2 u[4], xv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u[q] = ldc(U + (size_t)(j + q * kGemvWaves) * n + row);
      xv[q] = ldc(x + j + q * kGemvWaves);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double2& a = (q & 1) ? a1 : a0;
      a.x += u[q].x * xv[q].x - u[q].y * xv[q].y;
      a.y += u[q].x * xv[q].y + u[q].y * xv[q].x;
    }
  }
  for (; j < m; j += kGemvWaves) {
    const double2 u = ldc(U + (size_t)j * n + row), xv = ldc(x + j);
    a0.x += u.x * xv.x - u.y * xv.y;
    a0.y += u.x * xv.y + u.y * xv.x;
  }
}

__global__ __launch_bounds__(kGemvWaves * 64) void gemv_step_kernel(const GemvDesc* __restrict__ descs) {
  const GemvDesc& D = descs[blockIdx.y];
  const int rc = blockIdx.z;
  if (rc >= D.r || D.n <= 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + lane;
  const int rr = min(row, D.n - 1);  // rows past n compute a copy of the last and store nothing
  __shared__ double2 part[kGemvWaves][64];
  double2 a0 = make_double2(0.0, 0.0), a1 = make_double2(0.0, 0.0);
  if (blockIdx.x * 64 < D.n) {
    gemv_cols(D.U1, D.x1 + (size_t)rc * D.m1, D.m1, D.n, rr, wave, a0, a1);
    gemv_cols(D.U2, D.x2 + (size_t)rc * D.m2, D.m2, D.n, rr, wave, a0, a1);
  }
  part[wave][lane] = make_double2(a0.x + a1.x, a0.y + a1.y);
  __syncthreads();
  if (wave == 0 && row < D.n) {
    double2 s = gld(D.g + (size_t)rc * D.n + row);
#pragma unroll
    for (int w = 0; w < kGemvWaves; ++w) {
      s.x -= part[w][lane].x;
      s.y -= part[w][lane].y;
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
// After the last step of a level: P' = P M1 for every step, in place in the
// panel columns of W (read by nothing else afterwards).  A step's update of
// the other rows is then Y -= P' Y(pivot rows), with no Z to form for them.
__global__ __launch_bounds__(256) void gje_premul_kernel(const GjeDesc* __restrict__ descs) {
  const GjeDesc& D = descs[blockIdx.z];
  const int n = D.n, sidx = blockIdx.y, k = sidx * kGjeNb;
  if (k >= n) return;
  const int nb = min(kGjeNb, n - k);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  const int r0 = blockIdx.x * 64 + wave * 16;
  if (r0 >= n) return;  // no barriers in this kernel
  const cplx* M1 = D.M1 + (size_t)sidx * kGjeNb * kGjeNb;
  cplx* W = D.W;
  double2 a[4], b[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int row = r0 + lr, kq = 4 * kk + lq;
    a[kk] = ldc(W + (uint32_t)((k + min(kq, nb - 1)) * n + min(row, n - 1)));  // M1 is zero past nb
    b[kk] = gld(M1 + (size_t)lr * kGjeNb + kq);  // M1[kq][lr], column-major
  }
  dvec4 t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk].x, b[kk].x, t1, 0, 0, 0);
    t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk].y, b[kk].y, t2, 0, 0, 0);
    t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk].x + a[kk].y, b[kk].x + b[kk].y, t3, 0, 0, 0);
  }
  if (lr < nb)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = r0 + lq + 4 * q;
      if (row < n) gst(W + (size_t)(k + lr) * n + row, make_double2(t1[q] - t2[q], t3[q] - t1[q] - t2[q]));
    }
}

// Right-hand-side replay: one workgroup per TC columns keeps its tile Y in
// LDS and applies every step to it.  Per step: (1) each wave reads the pivot
// rows (from the rows that held the pivots, so before the interchanges) as
// its MFMA B operand, and the interchanges that move rows below the pivot
// block read their sources; (2) those rows are written; (3) the pivot block
// receives Z = M1 Y(pivot rows) and every other row Y -= P' Y(pivot rows).
// The multipliers of a wave's row blocks for the next step load while the
// current step runs.  Complex products take three real MFMA products.
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
    // eight loads in flight per thread (clamped addresses, no guarding branch)
    for (int e0 = tid; e0 < n * TC; e0 += kRhsWaves * 64 * 8) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = min(e0 + kRhsWaves * 64 * u, n * TC - 1);
        v[u] = ldc(W + (uint32_t)((c0 + min(e / n, nc - 1)) * n + e % n));
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + kRhsWaves * 64 * u;
        if (e < n * TC) Y[e % n][e / n] = e / n < nc ? v[u] : make_double2(0.0, 0.0);
      }
    }
    const int nsteps = min(s1, (n + kGjeNb - 1) / kGjeNb);
    // multipliers P' of a step for this wave's first PF row blocks
    // (lane: row r0 + lr, column 4 kk + lq)
    double2 pa[PF][4];
    auto load_p = [&](int sidx, int j, double2* dst) {
      const int k = sidx * kGjeNb, nb = min(kGjeNb, n - k);
      const int row = (wave + j * kRhsWaves) * 16 + lr;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int kq = 4 * kk + lq;
        // clamped: rows past n are not stored, columns past nb meet zero pivot rows
        dst[kk] = ldc(W + (uint32_t)((k + min(kq, nb - 1)) * n + min(row, n - 1)));
      }
    };
    // this lane's part of a step's interchange record, loaded a step ahead:
    // the rows holding pivots 4 kk + lq, the pair count and pair tid / TC
    struct PivInfo {
      int prow[4], naff, pd, ps;
    };
    auto load_piv = [&](int sidx, PivInfo& pi) {
      const auto piv = gmem(D.piv + (size_t)sidx * kGjePivStride);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) pi.prow[kk] = piv[1 + 4 * kGjeNb + 4 * kk + lq];
      pi.naff = piv[0];
      const int t = min(tid / TC, 2 * kGjeNb - 1);
      pi.pd = piv[1 + t];
      pi.ps = piv[1 + 2 * kGjeNb + t];
    };
    PivInfo pcur;
    if (s0 < nsteps) {
      load_piv(s0, pcur);
#pragma unroll
      for (int j = 0; j < PF; ++j) load_p(s0, j, pa[j]);
    }
    __syncthreads();
    for (int sidx = s0; sidx < nsteps; ++sidx) {
      const int k = sidx * kGjeNb;
      const int nb = min(kGjeNb, n - k);
      const PivInfo pi = pcur;
      if (sidx + 1 < nsteps) load_piv(sidx + 1, pcur);
      // 1. the pivot rows as the B operand (lane: row 4 kk + lq, column lr)
      double2 yb[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int q = 4 * kk + lq;
        yb[kk] = (q < nb && cl) ? Y[pi.prow[kk]][lr] : make_double2(0.0, 0.0);
      }
      const bool owner = ((k / 16) % kRhsWaves) == wave;  // this wave holds the pivot block
      double2 ma[4];
      if (owner) {
        const cplx* M1 = D.M1 + (size_t)sidx * kGjeNb * kGjeNb;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) ma[kk] = gld(M1 + (size_t)(4 * kk + lq) * kGjeNb + lr);  // M1[lr][4 kk + lq]
      }
      //    interchanged rows that land below the pivot block
      int dA = -1;
      double2 vA = make_double2(0.0, 0.0);
      if (tid < pi.naff * TC && pi.pd >= k + nb) {
        dA = pi.pd;
        vA = Y[pi.ps][tid % TC];
      }
      __syncthreads();
      // 2.
      if (dA >= 0) Y[dA][tid % TC] = vA;
      __syncthreads();
      // 3.
      double ys[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) ys[kk] = yb[kk].x + yb[kk].y;
#pragma unroll
      for (int j = 0; j < NBLK; ++j) {
        const int r0 = (wave + j * kRhsWaves) * 16;
        if (r0 >= n) break;
        dvec4 t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
        if (r0 == k) {  // Z = M1 Y(pivot rows)
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[kk].x, yb[kk].x, t1, 0, 0, 0);
            t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[kk].y, yb[kk].y, t2, 0, 0, 0);
            t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[kk].x + ma[kk].y, ys[kk], t3, 0, 0, 0);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = r0 + lq + 4 * q;
            if (cl && row < n) Y[row][lr] = make_double2(t1[q] - t2[q], t3[q] - t1[q] - t2[q]);
          }
        } else {
          double2 pb[4];
          if (j < PF) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) pb[kk] = pa[j < PF ? j : 0][kk];
          } else {
            load_p(sidx, j, pb);
          }
          // with every block's multipliers prefetched there are registers
          // for the block's old values: read before the products at clamped
          // indices (inside the tile; rows past n and columns past TC are
          // not stored), so the wave does not wait on LDS row by row after
          constexpr bool kEarly = PF == NBLK;
          double2 yo[4];
          if (kEarly) {
#pragma unroll
            for (int q = 0; q < 4; ++q) yo[q] = Y[min(r0 + lq + 4 * q, n - 1)][min(lr, TC - 1)];
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(pb[kk].x, yb[kk].x, t1, 0, 0, 0);
            t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(pb[kk].y, yb[kk].y, t2, 0, 0, 0);
            t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(pb[kk].x + pb[kk].y, ys[kk], t3, 0, 0, 0);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = r0 + lq + 4 * q;
            if (cl && row < n) {
              const double2 y = kEarly ? yo[q] : Y[row][lr];
              Y[row][lr] = make_double2(y.x - (t1[q] - t2[q]), y.y - (t3[q] - t1[q] - t2[q]));
            }
          }
        }
        if (j < PF && sidx + 1 < nsteps) load_p(sidx + 1, j, pa[j < PF ? j : 0]);
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

// Register-resident replay for orders above kRhsMaxN16 (up to kGjeMaxN):
// a 16-column tile of such an order does not fit in LDS, but it does fit in
// the registers of eight wavefronts, two per SIMD (256 registers each).
// Wave w holds the 16-row blocks w, w + 8, ... (up to 8 of them) of the tile
// in the matrix-core accumulator layout, real and imaginary parts apart:
// register q of lane (lq, lr) is row r0 + lq + 4 q of column lr.  So all 16
// lanes of a column do useful products (the LDS tile of these orders only
// had room for 8 or 10 columns) and the tile never passes through LDS.  Per
// step:
//   (0) one wave enters the step's pivot rows, the sources of the rows the
//       interchanges move below the pivot block and their destinations in
//       two row maps in LDS (tagged with the step, double-buffered);
//   (1) every lane looks up its own 32 rows (all 16 lanes of a row read
//       the same entry) and writes those the map names to an LDS stage
//       (double-buffered over steps), so no register of the tile is ever
//       picked by a runtime index;
//   (2) every wave reads the pivot rows as its B operand, the owners of
//       interchange destinations take their new values from the stage;
//   (3) the pivot block becomes M1 Y(pivot rows), every other block
//       Y -= P' Y(pivot rows), three real products per complex one; the
//       multipliers of the next block load while the current block's
//       products run (scheduling barriers every second block keep the
//       compiler from hoisting more loads than the register budget holds).
// The step's interchange record is read one step ahead, one entry per lane.
// Two barriers per step: after the maps, after the stage.
constexpr int kRegWaves = 8;
constexpr int kRegBlk = kGjeMaxN / 16 / kRegWaves;  // 8 row blocks per wave
constexpr int kRegAhead = 1;                         // multiplier blocks in flight
static_assert(kGjeNb == 16, "the register replay's pivot block of step k is row block k >> 4");

__global__ __launch_bounds__(kRegWaves * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void gje_rhs_reg_kernel(
    const GjeDesc* __restrict__ descs, int nbatch, int tiles_per, int s0, int s1) {
  constexpr int TC = 16;
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  // stage slots: 16 pivot rows, then up to 2 NB interchange sources
  __shared__ double2 stage[2][3 * kGjeNb][TC];
  // a step's rows, double-buffered over steps: smap[r] = 64 (s + 1) + slot
  // when step s stages row r into that slot (its pivot rows and the sources
  // of the rows moved below the pivot block), dmap[r] likewise when row r
  // takes its new value from the slot; entries of earlier steps carry a
  // smaller tag, so they need no clearing within a tile
  __shared__ unsigned short smap[2][kGjeMaxN], dmap[2][kGjeMaxN];
  for (int tile = blockIdx.x; tile < nbatch * tiles_per; tile += gridDim.x) {
    const GjeDesc& D = descs[tile / tiles_per];
    const int n = D.n;
    const int c0 = n + (tile % tiles_per) * TC;
    if (c0 >= D.ncol) continue;
    const int nc = min(TC, D.ncol - c0);
    cplx* W = D.W;
    dvec4 Yr[kRegBlk], Yi[kRegBlk];
    {
      const int col = c0 + min(lr, nc - 1);  // clamped: columns past nc are not stored
#pragma unroll
      for (int j = 0; j < kRegBlk; ++j) {
        const int r0 = (wave + j * kRegWaves) * 16;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double2 v = ldc(W + (uint32_t)(col * n + min(r0 + lq + 4 * q, n - 1)));
          Yr[j][q] = v.x;
          Yi[j][q] = v.y;
        }
      }
    }
    for (int i = tid; i < 2 * kGjeMaxN; i += kRegWaves * 64) {
      (&smap[0][0])[i] = 0;
      (&dmap[0][0])[i] = 0;
    }
    __syncthreads();
    const int nsteps = min(s1, (n + kGjeNb - 1) / kGjeNb);
    // interchange record of a step: lane t holds entry 1 + t (destinations
    // 0..31, then sources 0..31) in ra and entry 65 + t (pivot rows) in rb
    auto load_rec = [&](int sidx, int& ra, int& rb, int& naff) {
      const auto piv = gmem(D.piv + (size_t)sidx * kGjePivStride);
      ra = piv[1 + lane];
      rb = piv[1 + 4 * kGjeNb + min(lane, kGjeNb - 1)];
      naff = piv[0];
    };
    // multipliers P' of step k for row block j (lane: row r0 + lr, column
    // 4 kk + lq); the pivot block takes M1 instead (lane: M1[lr][4 kk + lq],
    // zero past nb), so that every block's operand is the one loaded ahead
    auto load_p = [&](int k, int nb, int j, double2* dst) {
      const int blk = wave + j * kRegWaves;
      const bool pv = blk == (k >> 4);  // uniform over the wave: a pointer select, no branch
      const cplx* M1 = D.M1 + (size_t)(k >> 4) * kGjeNb * kGjeNb + lr;
      const int row = min(blk * 16 + lr, n - 1);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        dst[kk] = ldc(pv ? M1 + (4 * kk + lq) * kGjeNb : W + (uint32_t)((k + min(4 * kk + lq, nb - 1)) * n + row));
    };
    int ra = 0, rb = 0, naff = 0;
    double2 pbuf[kRegAhead + 1][4];
    if (s0 < nsteps) {
      load_rec(s0, ra, rb, naff);
#pragma unroll
      for (int j = 0; j < kRegAhead; ++j) load_p(s0 * kGjeNb, min(kGjeNb, n - s0 * kGjeNb), j, pbuf[j]);
    }
    for (int sidx = s0; sidx < nsteps; ++sidx) {
      const int k = sidx * kGjeNb;
      const int nb = min(kGjeNb, n - k);
      const int cra = ra, crb = rb, cnaff = min(__builtin_amdgcn_readfirstlane(naff), 2 * kGjeNb);
      if (sidx + 1 < nsteps) load_rec(sidx + 1, ra, rb, naff);
      const int buf = sidx & 1;
      const int tag = 64 * (sidx + 1);
      __builtin_amdgcn_sched_barrier(0);
      // (0) wave 0 enters the step's rows in the maps: pivot c (lane c), and
      //     pair t (lane t: destination; lane 2 NB + t: source) when its
      //     destination lies below the pivot block
      if (wave == 0) {
        const int src = __shfl(cra, min(lane + 2 * kGjeNb, 63), 64);
        if (lane < nb && (unsigned)crb < (unsigned)n) smap[buf][crb] = (unsigned short)(tag + lane);
        if (lane < cnaff && cra >= k + nb && cra < n && (unsigned)src < (unsigned)n) {
          smap[buf][src] = (unsigned short)(tag + kGjeNb + lane);
          dmap[buf][cra] = (unsigned short)(tag + kGjeNb + lane);
        }
      }
      __syncthreads();
      // (1) every lane stages those of its rows that the map names
#pragma unroll
      for (int j = 0; j < kRegBlk; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int v = smap[buf][(wave + j * kRegWaves) * 16 + lq + 4 * q];
          if (v >= tag) stage[buf][v - tag][lr] = make_double2(Yr[j][q], Yi[j][q]);
        }
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
      // (2) the pivot rows as the B operand (lane: row 4 kk + lq, column lr),
      //     and their sums for the three-product form; interchange
      //     destinations below the block
      double yr[4], yi[4], ys[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double2 v = 4 * kk + lq < nb ? stage[buf][4 * kk + lq][lr] : make_double2(0.0, 0.0);
        yr[kk] = v.x;
        yi[kk] = v.y;
        ys[kk] = v.x + v.y;
      }
#pragma unroll
      for (int j = 0; j < kRegBlk; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int v = dmap[buf][(wave + j * kRegWaves) * 16 + lq + 4 * q];
          if (v >= tag) {
            const double2 y = stage[buf][v - tag][lr];
            Yr[j][q] = y.x;
            Yi[j][q] = y.y;
          }
        }
      // (3) products, three real ones per complex one, block by block, the
      //     multipliers kRegAhead blocks ahead in flight
      const int pblk = k >> 4;  // the pivot block
#pragma unroll
      for (int j = 0; j < kRegBlk; ++j) {
        if ((j & 1) == 0) __builtin_amdgcn_sched_barrier(0);
        const int blk = wave + j * kRegWaves;
        if (j + kRegAhead < kRegBlk) load_p(k, nb, j + kRegAhead, pbuf[(j + kRegAhead) % (kRegAhead + 1)]);
        if (blk * 16 >= n) continue;
        const double2* a = pbuf[j % (kRegAhead + 1)];
        const bool piv = blk == pblk;  // Z = M1 Y(pivot rows), a holding M1
        dvec4 t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk].x, yr[kk], t1, 0, 0, 0);
          t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk].y, yi[kk], t2, 0, 0, 0);
          t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk].x + a[kk].y, ys[kk], t3, 0, 0, 0);
        }
        if (piv) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            Yr[j][q] = t1[q] - t2[q];
            Yi[j][q] = t3[q] - t1[q] - t2[q];
          }
        } else {  // Y -= P' Y(pivot rows)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            Yr[j][q] -= t1[q] - t2[q];
            Yi[j][q] -= t3[q] - t1[q] - t2[q];
          }
        }
      }
      if (sidx + 1 < nsteps) {
#pragma unroll
        for (int j = 0; j < kRegAhead; ++j) load_p(k + kGjeNb, min(kGjeNb, n - k - kGjeNb), j, pbuf[j]);
      }
    }
    if (lr < nc) {
#pragma unroll
      for (int j = 0; j < kRegBlk; ++j) {
        const int r0 = (wave + j * kRegWaves) * 16;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = r0 + lq + 4 * q;
          if (row < n) gst(W + (size_t)(c0 + lr) * n + row, make_double2(Yr[j][q], Yi[j][q]));
        }
      }
    }
    __syncthreads();  // the next tile's first step may write the stage buffer read last
  }
}

void gje_init() {}

void launch_gje_panel(const GjeDesc* d, int nbatch, int k, int max_n, hipStream_t st) {
  if (nbatch <= 0 || max_n <= k) return;
  if (max_n - k <= 768)
    hipLaunchKernelGGL((gje_panel_kernel<768, 1>), dim3(nbatch), dim3(768), 0, st, d, k);
  else
    hipLaunchKernelGGL((gje_panel_kernel<512, 2>), dim3(nbatch), dim3(512), 0, st, d, k);
}
bool gje_step_fits(int max_n) { return max_n <= kUpdMaxN; }
// widest column range of an update of step k from column min(k + 16 + lo, n)
// on: the diagonal block, or with max_col > 0 the right-hand sides too (a
// matrix of order below k + 16 + lo starts at its own n)
static int update_width(int k, int max_n, int lo, int hi, int max_col, int max_rhs) {
  if (max_col <= 0) return std::min(max_n - k - kGjeNb, hi) - lo;
  return std::max(max_col - std::min(k + kGjeNb + lo, max_n), max_rhs);
}
int gje_step_max_blocks(int nbatch, int max_n, int max_col, int max_rhs) {
  const int width = update_width(0, max_n, kGjeNb, 1 << 30, max_col, max_rhs);  // the update of step 0
  return nbatch * (1 + (width > 0 ? (width - 1) / kUpdCols + 1 : 0));
}
void launch_gje_step(const GjeDesc* d, int nbatch, int k, int max_n, hipStream_t st, int max_col, int max_rhs) {
  if (nbatch <= 0 || max_n <= k) return;
  // update of step k - 16: columns [k + 16, max_n), and the right-hand sides
  const int width = k > 0 ? update_width(k - kGjeNb, max_n, kGjeNb, 1 << 30, max_col, max_rhs) : 0;
  const int utiles = width > 0 ? (width - 1) / kUpdCols + 1 : 0;
  hipLaunchKernelGGL(gje_step_kernel, dim3(nbatch * (1 + utiles)), dim3(kUpdWaves * 64), 0, st, d, nbatch, k,
                     utiles > 0 ? utiles : 1, max_col > 0 ? 1 : 0);
}
void launch_gje_update(const GjeDesc* d, int nbatch, int k, int max_n, int lo, int hi, hipStream_t st, int max_col,
                       int max_rhs) {
  const int width = update_width(k, max_n, lo, hi, max_col, max_rhs);
  if (nbatch > 0 && width > 0) {
    if (max_n <= kUpdMaxN) {
      const int tiles = (width - 1) / kUpdCols + 1;
      hipLaunchKernelGGL(gje_update_kernel, dim3(tiles, nbatch), dim3(kUpdWaves * 64), 0, st, d, k, lo, hi,
                         max_col > 0 ? 1 : 0);
    } else {  // the diagonal block only: callers pass max_col > 0 only where gje_step_fits holds
      const int tiles = (width - 1) / kUpdWideCols + 1;
      hipLaunchKernelGGL(gje_update_wide_kernel, dim3(tiles, nbatch), dim3(kUpdWideThreads), 0, st, d, k, lo, hi);
    }
  }
}
void launch_gje_premul(const GjeDesc* d, int nbatch, int max_n, hipStream_t st) {
  if (nbatch > 0 && max_n > 0)
    hipLaunchKernelGGL(gje_premul_kernel, dim3((max_n + 63) / 64, (max_n + kGjeNb - 1) / kGjeNb, nbatch), dim3(256),
                       0, st, d);
}
void launch_gje_rhs(const GjeDesc* d, int nbatch, int max_rhs, int max_n, int s0, int s1, int max_blocks,
                    hipStream_t st, bool narrow) {
  if (nbatch <= 0 || max_rhs <= 0 || s1 <= s0) return;
  // column tile: 16 (unless narrow), in LDS up to order kRhsMaxN16 and in
  // registers above; narrow: as many columns as the 160 KiB of LDS hold,
  // 8 up to order kRhsMaxN16, 10 up to kRhsMaxN10, 8 above
  const bool big = max_n > kRhsMaxN16;
  const int tc = !narrow ? 16 : (big && max_n <= kRhsMaxN10 ? 10 : 8);
  const int tiles_per = (max_rhs + tc - 1) / tc;
  const int total = nbatch * tiles_per;
  const int grid = max_blocks > 0 ? std::min(total, max_blocks) : total;
  if (tc == 16 && big)
    hipLaunchKernelGGL(gje_rhs_reg_kernel, dim3(grid), dim3(kRegWaves * 64), 0, st, d, nbatch, tiles_per, s0, s1);
  else if (tc == 16)
    hipLaunchKernelGGL((gje_rhs_kernel<16, kRhsMaxN16>), dim3(grid), dim3(kRhsWaves * 64), 0, st, d, nbatch,
                       tiles_per, s0, s1);
  else if (tc == 10)
    hipLaunchKernelGGL((gje_rhs_kernel<10, kRhsMaxN10>), dim3(grid), dim3(kRhsWaves * 64), 0, st, d, nbatch,
                       tiles_per, s0, s1);
  else
    hipLaunchKernelGGL((gje_rhs_kernel<8, kGjeMaxN>), dim3(grid), dim3(kRhsWaves * 64), 0, st, d, nbatch, tiles_per,
                       s0, s1);
}
void launch_gemv_step(const GemvDesc* d, int nbatch, int max_n, int max_r, hipStream_t st) {
  if (nbatch > 0 && max_n > 0 && max_r > 0)
    hipLaunchKernelGGL(gemv_step_kernel, dim3((max_n + 63) / 64, nbatch, max_r), dim3(kGemvWaves * 64), 0, st,
                       d);
}

}  // namespace mlh

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
//                      panel rows k..n-1 held in registers; writes the NB pivot rows, the
//                      inverse M1 of the NB x NB pivot block, and the
//                      multipliers P of rows >= k (L21 U11, the pivoted
//                      original panel values; zero on the pivot rows).  Rows
//                      above k use their current panel values, read from W;
//   gje_update_kernel  one workgroup per 32 trailing columns: applies the row
//                      swaps, Z = M1 Y(pivot rows), Y(other rows) -= P Z on the
//                      FP64 matrix cores, Y(pivot rows) = Z.
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

// Panel kernel: the (n - k) x NB tall panel lives in registers, thread t owning
// local rows t and t + 512 (n <= 608).
constexpr int kPanelThreads = 512;
constexpr int kUpdThreads = 1024;
constexpr int kUpdWaves = kUpdThreads / 64;
constexpr int kPanelSlots = (kGjeMaxN + kPanelThreads - 1) / kPanelThreads;

__global__ __launch_bounds__(kPanelThreads) void gje_panel_kernel(const GjeDesc* __restrict__ descs, int k) {
  const GjeDesc& D = descs[blockIdx.x];
  const int n = D.n;
  if (k >= n) return;
  const int nb = min(kGjeNb, n - k);
  const int L = n - k;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  cplx* W = D.W;
  __shared__ double bval[kPanelThreads / 64];
  __shared__ int bidx[kPanelThreads / 64];
  __shared__ double2 rowc[kGjeNb], rowp[kGjeNb];
  __shared__ int spiv[kGjeNb];
  __shared__ double2 lu11[kGjeNb][kGjeNb + 1];
  double2 a[kPanelSlots][kGjeNb];
#pragma unroll
  for (int sl = 0; sl < kPanelSlots; ++sl) {
    const int lr = tid + sl * kPanelThreads;
#pragma unroll
    for (int j = 0; j < kGjeNb; ++j)
      a[sl][j] = (lr < L && j < nb) ? gld(W + (size_t)(k + j) * n + k + lr) : make_double2(0.0, 0.0);
  }
  int singular = 0;
  for (int c = 0; c < nb; ++c) {
    double best = -1.0;
    int bi = c;
#pragma unroll
    for (int sl = 0; sl < kPanelSlots; ++sl) {
      const int lr = tid + sl * kPanelThreads;
      double2 v = make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < kGjeNb; ++j)
        if (j == c) v = a[sl][j];
      const double m2 = v.x * v.x + v.y * v.y;
      if (lr >= c && lr < L && m2 > best) {
        best = m2;
        bi = lr;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      bval[wave] = best;
      bidx[wave] = bi;
    }
    __syncthreads();
    double b = bval[0];
    int p = bidx[0];
#pragma unroll
    for (int w = 1; w < kPanelThreads / 64; ++w)
      if (bval[w] > b || (bval[w] == b && bidx[w] < p)) {
        b = bval[w];
        p = bidx[w];
      }
    if (tid == 0) spiv[c] = k + p;
    if (b <= 0.0 && singular == 0) singular = k + c + 1;
    // exchange rows c and p through LDS
    const int owner_p = p % kPanelThreads, slot_p = p / kPanelThreads;
    if (tid == c) {
#pragma unroll
      for (int j = 0; j < kGjeNb; ++j) rowc[j] = a[0][j];
    }
    if (tid == owner_p) {
#pragma unroll
      for (int sl = 0; sl < kPanelSlots; ++sl)
        if (sl == slot_p)
#pragma unroll
          for (int j = 0; j < kGjeNb; ++j) rowp[j] = a[sl][j];
    }
    __syncthreads();
    if (tid == owner_p) {
#pragma unroll
      for (int sl = 0; sl < kPanelSlots; ++sl)
        if (sl == slot_p)
#pragma unroll
          for (int j = 0; j < kGjeNb; ++j) a[sl][j] = rowc[j];
    }
    if (tid == c) {
#pragma unroll
      for (int j = 0; j < kGjeNb; ++j) a[0][j] = rowp[j];
    }
    // eliminate below the pivot with the new pivot row (= old row p, in LDS)
    const double2 ucc = rowp[c];
    const bool ok = (ucc.x != 0.0 || ucc.y != 0.0);
    const double2 ip = ok ? cinv2(ucc) : make_double2(0.0, 0.0);
#pragma unroll
    for (int sl = 0; sl < kPanelSlots; ++sl) {
      const int lr = tid + sl * kPanelThreads;
      if (lr > c && lr < L) {
        double2 l = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < kGjeNb; ++j)
          if (j == c) l = cmul2(a[sl][j], ip);
#pragma unroll
        for (int j = 0; j < kGjeNb; ++j) {
          if (j == c) a[sl][j] = l;
          if (j > c) {
            const double2 t = cmul2(l, rowp[j]);
            a[sl][j].x -= t.x;
            a[sl][j].y -= t.y;
          }
        }
      }
    }
  }
  if (tid == 0 && singular != 0) atomicCAS(D.info, 0, singular);
  // compose the NB row interchanges into (destination, source) pairs for the
  // update kernel: piv[0] = count, piv[1..] destinations, piv[1+2NB..] sources
  if (tid == 0) {
    int rows[2 * kGjeNb], from[2 * kGjeNb], na = 0;
    for (int q = 0; q < nb; ++q) {
      const int r1 = k + q, r2 = spiv[q];
      if (r1 == r2) continue;
      int i1 = -1, i2 = -1;
      for (int t = 0; t < na; ++t) {
        if (rows[t] == r1) i1 = t;
        if (rows[t] == r2) i2 = t;
      }
      if (i1 < 0) {
        rows[na] = r1;
        from[na] = r1;
        i1 = na++;
      }
      if (i2 < 0) {
        rows[na] = r2;
        from[na] = r2;
        i2 = na++;
      }
      const int t = from[i1];
      from[i1] = from[i2];
      from[i2] = t;
    }
    D.piv[0] = na;
    for (int t = 0; t < na; ++t) {
      D.piv[1 + t] = rows[t];
      D.piv[1 + 2 * kGjeNb + t] = from[t];
    }
  }
  // the pivot block L11\U11 sits in rows 0..nb-1 (threads 0..nb-1, slot 0)
  if (tid < kGjeNb) {
#pragma unroll
    for (int j = 0; j < kGjeNb; ++j) lu11[tid][j] = (tid < nb) ? a[0][j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // multipliers of the rows below the pivot block: P = L21 U11
#pragma unroll
  for (int sl = 0; sl < kPanelSlots; ++sl) {
    const int lr = tid + sl * kPanelThreads;
    if (lr < L) {
#pragma unroll
      for (int j = 0; j < kGjeNb; ++j) {
        double2 v = make_double2(0.0, 0.0);
        if (lr >= nb && j < nb) {
#pragma unroll
          for (int q = 0; q <= j; ++q) {
            const double2 t = cmul2(a[sl][q], lu11[q][j]);
            v.x += t.x;
            v.y += t.y;
          }
        }
        gst(D.P + (size_t)j * n + k + lr, v);
      }
    }
  }
  // M1 = (L11 U11)^{-1}, one thread per column, the column in registers
  // (fully unrolled so that only the 16 x 16 factors are read from LDS)
  if (tid < kGjeNb) {
    double2 x[kGjeNb];
#pragma unroll
    for (int r = 0; r < kGjeNb; ++r) x[r] = make_double2(r == tid ? 1.0 : 0.0, 0.0);
#pragma unroll
    for (int r = 1; r < kGjeNb; ++r)
#pragma unroll
      for (int q = 0; q < r; ++q) {
        const double2 t = cmul2(lu11[r][q], x[q]);
        x[r].x -= t.x;
        x[r].y -= t.y;
      }
#pragma unroll
    for (int r = kGjeNb - 1; r >= 0; --r) {
#pragma unroll
      for (int q = r + 1; q < kGjeNb; ++q) {
        const double2 t = cmul2(lu11[r][q], x[q]);
        x[r].x -= t.x;
        x[r].y -= t.y;
      }
      const double2 d = lu11[r][r];
      x[r] = (r < nb && (d.x != 0.0 || d.y != 0.0)) ? cmul2(x[r], cinv2(d)) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < kGjeNb; ++r) gst(D.M1 + (size_t)tid * kGjeNb + r, (tid < nb) ? x[r] : make_double2(0.0, 0.0));
  }

}

__global__ __launch_bounds__(kUpdThreads) void gje_update_kernel(const GjeDesc* __restrict__ descs, int k) {
  const GjeDesc& D = descs[blockIdx.y];
  const int n = D.n;
  if (k >= n) return;
  const int nb = min(kGjeNb, n - k);
  const int c0 = k + nb + blockIdx.x * kGjeCols;
  if (c0 >= D.ncol) return;
  const int nc = min(kGjeCols, D.ncol - c0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  cplx* W = D.W;
  __shared__ double zr[kGjeNb][kGjeCols + 1], zi[kGjeNb][kGjeCols + 1];
  __shared__ double2 m1[kGjeNb][kGjeNb];
  __shared__ double2 y1[kGjeNb][kGjeCols];
  // 1. row interchanges of this step on our columns, as (destination, source)
  //    pairs composed by the panel kernel: stage the sources, then write back
  __shared__ int sdst[2 * kGjeNb], ssrc[2 * kGjeNb];
  __shared__ double2 stage[2 * kGjeNb][kGjeCols];
  const int naff = D.piv[0];
  if (tid < naff) {
    sdst[tid] = D.piv[1 + tid];
    ssrc[tid] = D.piv[1 + 2 * kGjeNb + tid];
  }
  for (int e = tid; e < kGjeNb * kGjeNb; e += kUpdThreads) m1[e % kGjeNb][e / kGjeNb] = gld(D.M1 + e);
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
        const int row = r0 + (lane & 15), kq = kk + (lane >> 4);
        double2 a = make_double2(0.0, 0.0);
        if (row < k)
          a = kq < nb ? gld(W + (size_t)(k + kq) * n + row) : make_double2(0.0, 0.0);
        else if (row < n)
          a = gld(D.P + (size_t)kq * n + row);
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

// y = g - U1 x1 - U2 x2, one workgroup per 64 rows, four wavefronts split the columns
__global__ __launch_bounds__(256) void gemv_step_kernel(const GemvDesc* __restrict__ descs) {
  const GemvDesc& D = descs[blockIdx.y];
  const int row = blockIdx.x * 64 + (threadIdx.x & 63);
  const int wave = threadIdx.x >> 6;
  __shared__ double2 part[4][64];
  double2 acc = make_double2(0.0, 0.0);
  if (row < D.n) {
    for (int j = wave; j < D.m1; j += 4) {
      const double2 u = gld(D.U1 + (size_t)j * D.n + row), x = gld(D.x1 + j);
      acc.x += u.x * x.x - u.y * x.y;
      acc.y += u.x * x.y + u.y * x.x;
    }
    for (int j = wave; j < D.m2; j += 4) {
      const double2 u = gld(D.U2 + (size_t)j * D.n + row), x = gld(D.x2 + j);
      acc.x += u.x * x.x - u.y * x.y;
      acc.y += u.x * x.y + u.y * x.x;
    }
  }
  part[wave][threadIdx.x & 63] = acc;
  __syncthreads();
  if (wave == 0 && row < D.n) {
    double2 s = gld(D.g + row);
    for (int w = 0; w < 4; ++w) {
      s.x -= part[w][threadIdx.x].x;
      s.y -= part[w][threadIdx.x].y;
    }
    gst(D.y + row, s);
  }
}

void gje_init() {}

void launch_gje_panel(const GjeDesc* d, int nbatch, int k, int max_n, hipStream_t st) {
  const size_t lds = (size_t)(max_n - k) * kGjeNb * sizeof(double2);
  (void)lds;
  if (nbatch > 0 && max_n > k) hipLaunchKernelGGL(gje_panel_kernel, dim3(nbatch), dim3(kPanelThreads), 0, st, d, k);
}
void launch_gje_update(const GjeDesc* d, int nbatch, int k, int max_ncol, hipStream_t st) {
  const int tiles = (max_ncol - k - 1) / kGjeCols + 1;
  if (nbatch > 0 && max_ncol > k)
    hipLaunchKernelGGL(gje_update_kernel, dim3(tiles, nbatch), dim3(kUpdThreads), 0, st, d, k);
}
void launch_gemv_step(const GemvDesc* d, int nbatch, int max_n, hipStream_t st) {
  if (nbatch > 0 && max_n > 0) hipLaunchKernelGGL(gemv_step_kernel, dim3((max_n + 63) / 64, nbatch), dim3(256), 0, st, d);
}

}  // namespace mlh

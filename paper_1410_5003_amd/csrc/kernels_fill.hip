// Fill kernels: every alpha-independent matrix piece of the discretised
// coupled system (Sec. 2.5; pieces as in the sweep precomputation of Sec. 3.4).
//
//  fill_kernel    plain Nystrom / proxy blocks: one thread per (target, source)
//                 pair, 64 consecutive targets per wave so that the
//                 column-major stores are coalesced.
//  self_kernel    self blocks A_ii (eq. (37)): difference kernels of layers i
//                 and i+1 over the three copies, zero inside the Alpert window
//                 |J - m| < a of the extended index J = j + l N, jump terms
//                 -I / +I on the diagonal.
//  alpert_kernel  the auxiliary-node correction inside the window (Sec. 2.5
//                 and the Remark on the quasi-periodic wrap): one wavefront per
//                 target row owns every corrected column of that row, so the
//                 read-modify-write needs no atomics.  On a cornered interface
//                 the window, the stencil and the correction stay inside the
//                 target's graded segment (cyclic in the segment parameter, no
//                 Bloch phase), and the interpolated quantity is the density
//                 times the graded Jacobian, so the stencil weights multiply
//                 the node weights w_j.
//  assemble_kernel  the blocks for one Bloch phase alpha as weighted sums of
//                 the pieces (Sec. 3.4), one workgroup per 2048 elements; the
//                 tile routine is shared with the least-squares panel
//                 launches, which carry the blocks of the block-tridiagonal
//                 system.
#include <algorithm>

#include "internal.hpp"

namespace mlh {

template <class T>
__device__ inline int find_job(const T* jobs, int njobs, int key) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile_begin <= key)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline void store(cplx* p, cplx v) { stc(p, v.re, v.im); }

// the self-block kernel K^{ka} - K^{kb} (dk = 0) or its derivative in ka
// (dk = 1: dK/dk at ka) or in kb (dk = 2: -dK/dk at kb)
__device__ inline Kern4 self_kern(int dk, double ka, double kb, double r2, double nd, double npd, double nn) {
  if (dk == 0) return lp_kernels_diff(ka, kb, r2, nd, npd, nn);
  Kern4 K = lp_kernels_dk(dk == 1 ? ka : kb, r2, nd, npd, nn);
  if (dk == 2) {
    K.S = {-K.S.re, -K.S.im};
    K.D = {-K.D.re, -K.D.im};
    K.Ds = {-K.Ds.re, -K.Ds.im};
    K.T = {-K.T.re, -K.T.im};
  }
  return K;
}

// Both neighbour blocks of a pair of curves from one Hankel evaluation per
// (m, j, copy): entry (m, j) of copy p and entry (j, m) of copy 2 - p have the
// same distance, and swapping target and source negates both normal
// projections, which leaves S and T and exchanges D with D*.  16 x 16 tiles,
// so that both blocks are written in runs of consecutive rows.
template <bool DK>
__device__ __forceinline__ void fill_pair(const FillJob& J, int lt) {
  const int tm = lt % J.tiles_m, tn = lt / J.tiles_m;
  const int m = tm * kSelfTile + (int)(threadIdx.x % kSelfTile);
  const int j = tn * kSelfTile + (int)(threadIdx.x / kSelfTile);
  if (m >= J.Mt || j >= J.Ns) return;
  const double tx = J.tx[m], ty = J.ty[m] + J.dy0, tnx = J.tnx[m], tny = J.tny[m];
  const double sx = J.sx[j], sy = J.sy[j], snx = J.snx[j], sny = J.sny[j];
  const double dy = ty - sy;
  const double nn = tnx * snx + tny * sny;
  const double w = J.sw[j] * J.scale, wt = J.tw[m] * J.scale_t;
  const int ld = J.ld, ldt = J.ld_t;
  for (int p = 0; p < J.npieces; ++p) {
    const double dx = (tx - sx) + (J.tshift[p] - J.sshift[p]);
    const double r2 = dx * dx + dy * dy;
    const Kern4 K = DK ? lp_kernels_dk(J.k, r2, tnx * dx + tny * dy, snx * dx + sny * dy, nn)
                       : lp_kernels(J.k, r2, tnx * dx + tny * dy, snx * dx + sny * dy, nn);
    cplx* o = J.out[p];
    store(o + (size_t)j * ld + m, {K.D.re * w, K.D.im * w});
    store(o + (size_t)(J.Ns + j) * ld + m, {K.S.re * w, K.S.im * w});
    store(o + (size_t)j * ld + J.Mt + m, {K.T.re * w, K.T.im * w});
    store(o + (size_t)(J.Ns + j) * ld + J.Mt + m, {K.Ds.re * w, K.Ds.im * w});
    cplx* q = J.out_t[J.npieces - 1 - p];
    store(q + (size_t)m * ldt + j, {K.Ds.re * wt, K.Ds.im * wt});
    store(q + (size_t)(J.Mt + m) * ldt + j, {K.S.re * wt, K.S.im * wt});
    store(q + (size_t)m * ldt + J.Ns + j, {K.T.re * wt, K.T.im * wt});
    store(q + (size_t)(J.Mt + m) * ldt + J.Ns + j, {K.D.re * wt, K.D.im * wt});
  }
}

// DK: the wavenumber-derivative pieces (jobs with dk set) instead of the pieces
template <bool DK>
__global__ __launch_bounds__(256) void fill_kernel(const FillJob* __restrict__ jobs, int njobs, int tile0) {
  const int tile = tile0 + (int)blockIdx.x;
  const FillJob& J = jobs[find_job(jobs, njobs, tile)];
  const int lt = tile - J.tile_begin;
  if (J.kind == kFillPair) {
    fill_pair<DK>(J, lt);
    return;
  }
  const int tm = lt % J.tiles_m, tn = lt / J.tiles_m;
  const int m = tm * kFillTileM + (threadIdx.x & (kFillTileM - 1));
  const int j = tn * kFillTileN + threadIdx.x / kFillTileM;
  if (m >= J.Mt || j >= J.Ns) return;
  const double tx = J.tx[m];
  const double ty = J.ty[m] + J.dy0;
  const double tnx = J.tnx ? J.tnx[m] : J.cnx;
  const double tny = J.tny ? J.tny[m] : J.cny;
  const double sx = J.sx[j], sy = J.sy[j], snx = J.snx[j], sny = J.sny[j];
  const double dy = ty - sy;
  const double nn = tnx * snx + tny * sny;
  const int ld = J.ld;
  for (int p = 0; p < J.npieces; ++p) {
    const double dx = (tx - sx) + (J.tshift[p] - J.sshift[p]);
    const double r2 = dx * dx + dy * dy;
    const double nd = tnx * dx + tny * dy;
    const double npd = snx * dx + sny * dy;
    cplx* o = J.out[p];
    if (DK && J.kind == kFillLayerPotential) {
      const Kern4 Kk = lp_kernels_dk(J.k, r2, nd, npd, nn);
      const double w = J.sw[j] * J.scale;
      store(o + (size_t)j * ld + m, {Kk.D.re * w, Kk.D.im * w});
      store(o + (size_t)(J.Ns + j) * ld + m, {Kk.S.re * w, Kk.S.im * w});
      store(o + (size_t)j * ld + J.Mt + m, {Kk.T.re * w, Kk.T.im * w});
      store(o + (size_t)(J.Ns + j) * ld + J.Mt + m, {Kk.Ds.re * w, Kk.Ds.im * w});
      continue;
    }
    const Kern4 K = lp_kernels(J.k, r2, nd, npd, nn);
    if (DK) {
      // d/dk of phi = D + i k S and of dphi/dn = T + i k D*
      const Kern4 Kk = lp_kernels_dk(J.k, r2, nd, npd, nn);
      const double k = J.k, s = J.scale;
      const cplx phi = {Kk.D.re - K.S.im - k * Kk.S.im, Kk.D.im + K.S.re + k * Kk.S.re};
      const cplx dphi = {Kk.T.re - K.Ds.im - k * Kk.Ds.im, Kk.T.im + K.Ds.re + k * Kk.Ds.re};
      store(o + (size_t)j * ld + m, {phi.re * s, phi.im * s});
      store(o + (size_t)j * ld + J.Mt + m, {dphi.re * s, dphi.im * s});
    } else if (J.kind == kFillLayerPotential) {
      const double w = J.sw[j] * J.scale;
      store(o + (size_t)j * ld + m, {K.D.re * w, K.D.im * w});
      store(o + (size_t)(J.Ns + j) * ld + m, {K.S.re * w, K.S.im * w});
      store(o + (size_t)j * ld + J.Mt + m, {K.T.re * w, K.T.im * w});
      store(o + (size_t)(J.Ns + j) * ld + J.Mt + m, {K.Ds.re * w, K.Ds.im * w});
    } else {
      // phi = dG/dn_p + i k G ; dphi/dn = T + i k D*   (eq. (15))
      const double k = J.k, s = J.scale;
      const cplx phi = {K.D.re - k * K.S.im, K.D.im + k * K.S.re};
      const cplx dphi = {K.T.re - k * K.Ds.im, K.T.im + k * K.Ds.re};
      store(o + (size_t)j * ld + m, {phi.re * s, phi.im * s});
      store(o + (size_t)j * ld + J.Mt + m, {dphi.re * s, dphi.im * s});
    }
  }
}

// Self blocks by pairs: entry (m, j) of copy l and entry (j, m) of copy -l
// have the same distance, so one Hankel evaluation serves both.  Swapping
// target and source negates both normal projections, which leaves S and T
// and exchanges D with D* (the source weight becomes w_m); the Alpert window
// is symmetric too.  Workgroups take the 16 x 16 blocks (bm, bn), bm <= bn,
// of the upper triangle; thread t the pair (bm 16 + t % 16, bn 16 + t / 16),
// and on a diagonal block only pairs with m <= j.
template <bool DK>
__global__ __launch_bounds__(256) void self_kernel(const SelfJob* __restrict__ jobs, int njobs, int a, int tile0) {
  const int tile = tile0 + (int)blockIdx.x;
  const SelfJob& J = jobs[find_job(jobs, njobs, tile)];
  const int lt = tile - J.tile_begin;
  int bn = (int)((sqrt(8.0 * lt + 1.0) - 1.0) * 0.5);  // lt = bn (bn + 1) / 2 + bm, bm <= bn
  while (bn * (bn + 1) / 2 > lt) --bn;
  while ((bn + 1) * (bn + 2) / 2 <= lt) ++bn;
  const int bm = lt - bn * (bn + 1) / 2;
  const int N = J.N;
  const int m = bm * kSelfTile + (int)(threadIdx.x % kSelfTile);
  const int j = bn * kSelfTile + (int)(threadIdx.x / kSelfTile);
  if (m >= N || j >= N || m > j) return;
  const double tnx = J.nx[m], tny = J.ny[m];
  const double snx = J.nx[j], sny = J.ny[j];
  const double dy = J.y[m] - J.y[j];
  const double dx0 = J.x[m] - J.x[j];
  const double nn = tnx * snx + tny * sny;
  const double wj = J.w[j], wm = J.w[m];
  const int ld = 2 * N;
  // Alpert window: smooth curves exclude |J - m| < a over the extended index
  // J = j + l N; a cornered curve excludes, in copy l = 0 only, the nodes of
  // the target's own segment within cyclic segment-local distance a
  bool same_seg = false;
  int cyc = 0;
  if (J.seg_lo) {
    same_seg = J.seg_lo[j] == J.seg_lo[m];
    const int len = J.seg_len[m];
    const int dd = j - m;
    cyc = dd < len - dd ? dd : len - dd;
  }
  for (int l = -1; l <= 1; ++l) {
    const int off = j + l * N - m;
    Kern4 K = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    const bool plain = J.seg_lo ? !(l == 0 && same_seg && cyc < a) : (off >= a || off <= -a);
    if (plain) {
      const double dx = dx0 - l * J.d;
      const double r2 = dx * dx + dy * dy;
      K = self_kern(DK ? J.dk : 0, J.ka, J.kb, r2, tnx * dx + tny * dy, snx * dx + sny * dy, nn);
    }
    // (m, j) of copy l, source weight w_j
    cplx D = {K.D.re * wj, K.D.im * wj}, S = {K.S.re * wj, K.S.im * wj};
    cplx T = {K.T.re * wj, K.T.im * wj}, Ds = {K.Ds.re * wj, K.Ds.im * wj};
    if (!DK && l == 0 && j == m) {  // jump relations: -tau / +sigma
      D.re -= 1.0;
      Ds.re += 1.0;
    }
    cplx* o = J.out[l + 1];
    store(o + (size_t)j * ld + m, D);
    store(o + (size_t)(N + j) * ld + m, S);
    store(o + (size_t)j * ld + N + m, T);
    store(o + (size_t)(N + j) * ld + N + m, Ds);
    if (j != m) {  // (j, m) of copy -l: D and D* exchanged, source weight w_m
      cplx* p = J.out[1 - l];
      store(p + (size_t)m * ld + j, {K.Ds.re * wm, K.Ds.im * wm});
      store(p + (size_t)(N + m) * ld + j, {K.S.re * wm, K.S.im * wm});
      store(p + (size_t)m * ld + N + j, {K.T.re * wm, K.T.im * wm});
      store(p + (size_t)(N + m) * ld + N + j, {K.D.re * wm, K.D.im * wm});
    }
  }
}

template <bool DK>
__global__ __launch_bounds__(64) void alpert_kernel(const AlpertJob* __restrict__ jobs, int njobs, int a, int blk0) {
  const int blk = blk0 + (int)blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_begin <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  const AlpertJob& J = jobs[lo];
  const int m = blk - J.block_begin;
  const int N = J.N;
  // cornered interface: work in the target's segment, cyclically, piece l = 0
  const bool seg = J.seg_lo != nullptr;
  const int s_lo = seg ? J.seg_lo[m] : 0;
  const int s_len = seg ? J.seg_len[m] : N;
  const int m_idx = seg ? m - s_lo : m;
  __shared__ cplx kv[kAlpertAux][4];
  __shared__ double tpos[kAlpertAux];
  __shared__ double invden[kAlpertStencil];  // 1 / prod_{s != r} (r - s) of the Lagrange basis
  const int lane = threadIdx.x;
  if (lane < kAlpertStencil) {
    double den = 1.0;  // an integer below 16!, exact in double
    for (int s = 0; s < kAlpertStencil; ++s)
      if (s != lane) den *= (double)(lane - s);
    invden[lane] = 1.0 / den;
  }
  if (lane < kAlpertAux) {
    const size_t q = (size_t)m * kAlpertAux + lane;
    const Kern4 K = self_kern(DK ? J.dk : 0, J.ka, J.kb, J.r2[q], J.nd[q], J.npd[q], J.nn[q]);
    const double c = J.cw[q];
    kv[lane][0] = {K.D.re * c, K.D.im * c};
    kv[lane][1] = {K.S.re * c, K.S.im * c};
    kv[lane][2] = {K.T.re * c, K.T.im * c};
    kv[lane][3] = {K.Ds.re * c, K.Ds.im * c};
    tpos[lane] = J.t[q];
  }
  __syncthreads();
  const int half = a + 8;
  if (lane > 2 * half) return;
  const int Jx = m_idx - half + lane;  // extended (or segment-local) column index
  cplx acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  bool any = false;
  for (int q = 0; q < kAlpertAux; ++q) {
    const double t = tpos[q];
    const int j0 = (int)floor(t) - (kAlpertStencil / 2 - 1);
    const int r = Jx - j0;
    if (r < 0 || r >= kAlpertStencil) continue;
    double L = invden[r];
    for (int s = 0; s < kAlpertStencil; ++s)
      if (s != r) L *= t - (double)(j0 + s);
    any = true;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[e].re += L * kv[q][e].re;
      acc[e].im += L * kv[q][e].im;
    }
  }
  if (!any) return;
  int l, col;
  if (seg) {  // 2 half + 1 <= s_len, so no two lanes share a column
    l = 0;
    col = s_lo + (Jx >= 0 ? Jx % s_len : (s_len - 1) - ((-Jx - 1) % s_len));
    const double wc = J.colw[col];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[e].re *= wc;
      acc[e].im *= wc;
    }
  } else {
    l = (Jx >= 0) ? Jx / N : -((-Jx + N - 1) / N);
    col = Jx - l * N;
  }
  cplx* o = J.out[l + 1];
  const int ld = 2 * N;
  const size_t idx[4] = {(size_t)col * ld + m, (size_t)(N + col) * ld + m, (size_t)col * ld + N + m,
                         (size_t)(N + col) * ld + N + m};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double2 v = *reinterpret_cast<double2*>(o + idx[e]);
    v.x += acc[e].re;
    v.y += acc[e].im;
    *reinterpret_cast<double2*>(o + idx[e]) = v;
  }
}

// one workgroup per kAsmTile elements of one job (jobs own whole tiles)
__global__ __launch_bounds__(256) void assemble_kernel(const AsmJob* __restrict__ jobs, int njobs, int tile0) {
  assemble_one<kAsmTile / 256>(jobs, njobs, tile0 + (int)blockIdx.x, (int)threadIdx.x);
}

__global__ void hankel_eval_kernel(const double* x, double* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cplx h0, g;
  hankel_pieces(x[i], h0, g);
  out[4 * i + 0] = h0.re;
  out[4 * i + 1] = h0.im;
  out[4 * i + 2] = g.re;
  out[4 * i + 3] = g.im;
}

// launches larger than kMaxLaunchBlocks workgroups are split, each part
// passing its first tile index
void launch_fill(const FillJob* d_jobs, int njobs, int total_tiles, hipStream_t st, bool dk) {
  for (int t0 = 0; t0 < total_tiles; t0 += kMaxLaunchBlocks) {
    if (dk)
      hipLaunchKernelGGL(fill_kernel<true>, dim3(std::min(kMaxLaunchBlocks, total_tiles - t0)), dim3(256), 0, st,
                         d_jobs, njobs, t0);
    else
      hipLaunchKernelGGL(fill_kernel<false>, dim3(std::min(kMaxLaunchBlocks, total_tiles - t0)), dim3(256), 0, st,
                         d_jobs, njobs, t0);
  }
}
void launch_self(const SelfJob* d_jobs, int njobs, int total_tiles, int a_excl, hipStream_t st, bool dk) {
  for (int t0 = 0; t0 < total_tiles; t0 += kMaxLaunchBlocks) {
    if (dk)
      hipLaunchKernelGGL(self_kernel<true>, dim3(std::min(kMaxLaunchBlocks, total_tiles - t0)), dim3(256), 0, st,
                         d_jobs, njobs, a_excl, t0);
    else
      hipLaunchKernelGGL(self_kernel<false>, dim3(std::min(kMaxLaunchBlocks, total_tiles - t0)), dim3(256), 0, st,
                         d_jobs, njobs, a_excl, t0);
  }
}
void launch_alpert(const AlpertJob* d_jobs, int njobs, int total_blocks, int a_excl, hipStream_t st, bool dk) {
  for (int b0 = 0; b0 < total_blocks; b0 += kMaxLaunchBlocks) {
    if (dk)
      hipLaunchKernelGGL(alpert_kernel<true>, dim3(std::min(kMaxLaunchBlocks, total_blocks - b0)), dim3(64), 0, st,
                         d_jobs, njobs, a_excl, b0);
    else
      hipLaunchKernelGGL(alpert_kernel<false>, dim3(std::min(kMaxLaunchBlocks, total_blocks - b0)), dim3(64), 0, st,
                         d_jobs, njobs, a_excl, b0);
  }
}
void launch_assemble(const AsmJob* d_jobs, int njobs, int total_tiles, hipStream_t st) {
  for (int t0 = 0; t0 < total_tiles; t0 += kMaxLaunchBlocks)
    hipLaunchKernelGGL(assemble_kernel, dim3(std::min(kMaxLaunchBlocks, total_tiles - t0)), dim3(256), 0, st, d_jobs,
                       njobs, t0);
}
void launch_hankel_eval(const double* x, double* out, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(hankel_eval_kernel, dim3((n + 255) / 256), dim3(256), 0, st, x, out, n);
}

}  // namespace mlh

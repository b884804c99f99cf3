// Adjoint of the summed zeroth-order reflected efficiency.
//
// The discrete system (eq. (67)) has density rows A eta + B c = f and, per
// layer j, wall and radiation rows C'_j eta + Q'_j x_j = 0 with x_j = [c_j;
// a_j].  The solve is a linear map from the right-hand side to the unknowns;
// the zeroth reflected amplitude is a0 = l^T r for the adjoint vector l of
// that map (Sec. 3.2-3.3 read backwards):
//   A'^T z = w,  w = the row of X_1 that gives a0 (on interface 1),
//   l_eta = -z,
//   l_w,j = (Q'_j^+)^T v_j,  v_j = B_j^T z (+ the unit vector of a0 in layer 1).
// A change dE of the blocks moves a0 by -l^T dE u (u the solution), so
//   dJ/dp = sum_theta 2 Re(conj(a0) (-l^T dE/dp u)).
//
//  transpose_kernel   one 32 x 32 tile of dst = src^T (src null: zeros); the
//                     transposed block-tridiagonal system and its
//                     right-hand side are written with it;
//  btz_kernel         v_j = B1^T z1 + B2^T z2 for one layer (transposes, not
//                     conjugates), plus the unit entry of a0;
//  ls_adjoint_kernel  l_w = (Q'^+)^T v for one layer from its Tikhonov QR
//                     [Q'; mu I] = Q_f R (the least-squares kernels' factors):
//                     Q'^+ = R^{-1} Q_f[0:m]^H, so l_w = conj(Q_f[0:m] conj(t))
//                     with R^T t = v (forward substitution) and Q_f applied
//                     as its block reflectors, last panel first;
//  bilinear_kernel    left^T (sum_p coef_p P_p) right over a 64 x 64 tile of
//                     one block of derivative pieces, summed into the
//                     block's accumulator.
#include "internal.hpp"

namespace mlh {

__global__ __launch_bounds__(256) void transpose_kernel(const TransposeJob* __restrict__ jobs, int njobs) {
  int lo = 0, hi = njobs - 1;
  const int tile = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile_begin <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  const TransposeJob& J = jobs[lo];
  const int lt = tile - J.tile_begin;
  const int tr = (J.rows + 31) / 32;
  const int r0 = (lt % tr) * 32, c0 = (lt / tr) * 32;
  __shared__ double2 t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  // src(c, r) for dst rows r0.. and cols c0..: read src row-major in c
  for (int q = ty; q < 32; q += 8) {
    const int r = r0 + tx, c = c0 + q;  // dst (r, c) = src (c, r) = src[c + r * lds]
    double2 v = make_double2(0.0, 0.0);
    if (J.src && r < J.rows && c < J.cols) v = ldc(J.src + (size_t)r * J.lds + c);
    t[q][tx] = v;
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int r = r0 + tx, c = c0 + q;
    if (r < J.rows && c < J.cols) stc(J.dst + (size_t)c * J.ldd + r, t[q][tx].x, t[q][tx].y);
  }
}

__global__ __launch_bounds__(256) void btz_kernel(const BtzJob* __restrict__ jobs) {
  const BtzJob& J = jobs[blockIdx.x];
  for (int p = threadIdx.x; p < J.c; p += 256) {
    double re = 0.0, im = 0.0;
    if (p < J.P) {
      for (int part = 0; part < 2; ++part) {
        const cplx* B = part ? J.B2 : J.B1;
        const cplx* z = part ? J.z2 : J.z1;
        const int n = part ? J.n2 : J.n1, ld = part ? J.ld2 : J.ld1;
        if (!B) continue;
        for (int r = 0; r < n; ++r) {
          const double2 b = ldc(B + (size_t)p * ld + r), x = ldc(z + r);
          re += b.x * x.x - b.y * x.y;
          im += b.x * x.y + b.y * x.x;
        }
      }
    }
    if (p == J.unit) re += 1.0;
    stc(J.v + p, re, im);
  }
}

__device__ inline double blk_sum(double v, double* red) {
  // sum over the 256 threads of the workgroup, returned in every thread
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void ls_adjoint_kernel(const LsAdjJob* __restrict__ jobs) {
  const LsAdjJob& J = jobs[blockIdx.x];
  const int M = J.M, m = J.m, c = J.c, tid = threadIdx.x;
  __shared__ double2 y[kHqMaxRows];
  __shared__ double red[4];
  __shared__ double2 w[kHqNb], w2[kHqNb];
  for (int r = tid; r < M; r += 256) y[r] = make_double2(0.0, 0.0);
  __syncthreads();
  // R^T t = v, t kept in y[0:c]
  for (int k = 0; k < c; ++k) {
    double dr = 0.0, di = 0.0;
    for (int i = tid; i < k; i += 256) {
      const double2 rr = ldc(J.S + (size_t)k * M + i), t = y[i];
      dr += rr.x * t.x - rr.y * t.y;
      di += rr.x * t.y + rr.y * t.x;
    }
    dr = blk_sum(dr, red);
    di = blk_sum(di, red);
    if (tid == 0) {
      const double2 v = ldc(J.v + k);
      const double rkk = ldc(J.S + (size_t)k * M + k).x;  // the real beta of the reflector
      y[k] = make_double2((v.x - dr) / rkk, (v.y - di) / rkk);
    }
    __syncthreads();
  }
  // s = conj(t) padded with zeros, then Q_f s = prod_p (I - V_p T_p V_p^H) s
  for (int r = tid; r < c; r += 256) y[r].y = -y[r].y;
  __syncthreads();
  const int np = (c + kHqNb - 1) / kHqNb;
  for (int p = np - 1; p >= 0; --p) {
    const int k0 = p * kHqNb, nb = min(kHqNb, c - k0);
    const cplx* T = J.T + (size_t)p * kHqNb * kHqNb;
    // w = V^H y
    for (int i = 0; i < nb; ++i) {
      double ar = 0.0, ai = 0.0;
      for (int r = k0 + i + tid; r < M; r += 256) {
        const double2 v = r == k0 + i ? make_double2(1.0, 0.0) : ldc(J.S + (size_t)(k0 + i) * M + r);
        const double2 x = y[r];
        ar += v.x * x.x + v.y * x.y;  // conj(v) x
        ai += v.x * x.y - v.y * x.x;
      }
      ar = blk_sum(ar, red);
      ai = blk_sum(ai, red);
      if (tid == 0) w[i] = make_double2(ar, ai);
    }
    __syncthreads();
    if (tid < nb) {
      double ar = 0.0, ai = 0.0;
      for (int b = 0; b < nb; ++b) {
        const double2 t = ldc(T + tid + kHqNb * b), x = w[b];
        ar += t.x * x.x - t.y * x.y;
        ai += t.x * x.y + t.y * x.x;
      }
      w2[tid] = make_double2(ar, ai);
    }
    __syncthreads();
    for (int r = k0 + tid; r < M; r += 256) {
      double ar = 0.0, ai = 0.0;
      for (int i = 0; i < nb && k0 + i <= r; ++i) {
        const double2 v = r == k0 + i ? make_double2(1.0, 0.0) : ldc(J.S + (size_t)(k0 + i) * M + r);
        const double2 x = w2[i];
        ar += v.x * x.x - v.y * x.y;
        ai += v.x * x.y + v.y * x.x;
      }
      y[r].x -= ar;
      y[r].y -= ai;
    }
    __syncthreads();
  }
  for (int r = tid; r < m; r += 256) stc(J.ell + r, y[r].x, -y[r].y);
}

constexpr int kBilinTile = 64;

__global__ __launch_bounds__(256) void bilinear_kernel(const BilinJob* __restrict__ jobs, int njobs,
                                                       double* __restrict__ acc) {
  int lo = 0, hi = njobs - 1;
  const int tile = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile_begin <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  const BilinJob& J = jobs[lo];
  const int lt = tile - J.tile_begin;
  const int tr = (J.rows + kBilinTile - 1) / kBilinTile;
  const int r0 = (lt % tr) * kBilinTile, c0 = (lt / tr) * kBilinTile;
  const int r = r0 + (threadIdx.x & 63);
  __shared__ double red[4];
  double sr = 0.0, si = 0.0;
  if (r < J.rows) {
    // this thread: row r, columns c0 + q for q = wave, wave + 4, ...
    double er = 0.0, ei = 0.0;  // sum_c E(r, c) right(c)
    for (int cc = c0 + (int)(threadIdx.x >> 6); cc < min(c0 + kBilinTile, J.cols); cc += 4) {
      double vr = 0.0, vi = 0.0;
      for (int p = 0; p < J.np; ++p) {
        const double2 e = ldc(J.P[p] + (size_t)cc * J.ld + r);
        vr += J.coef[p].re * e.x - J.coef[p].im * e.y;
        vi += J.coef[p].re * e.y + J.coef[p].im * e.x;
      }
      const double2 x = ldc(J.right + cc);
      er += vr * x.x - vi * x.y;
      ei += vr * x.y + vi * x.x;
    }
    const double2 l = ldc(J.left + r);
    sr = l.x * er - l.y * ei;
    si = l.x * ei + l.y * er;
  }
  sr = blk_sum(sr, red);
  si = blk_sum(si, red);
  if (threadIdx.x == 0) {
    atomicAdd(acc + 2 * J.out, J.scale * sr);
    atomicAdd(acc + 2 * J.out + 1, J.scale * si);
  }
}

void launch_transpose(const TransposeJob* d, int njobs, int tiles, hipStream_t st) {
  for (int t0 = 0; t0 < tiles; t0 += kMaxLaunchBlocks)
    if (njobs > 0)
      hipLaunchKernelGGL(transpose_kernel, dim3(std::min(kMaxLaunchBlocks, tiles - t0)), dim3(256), 0, st, d, njobs);
}
void launch_btz(const BtzJob* d, int njobs, hipStream_t st) {
  if (njobs > 0) hipLaunchKernelGGL(btz_kernel, dim3(njobs), dim3(256), 0, st, d);
}
void launch_ls_adjoint(const LsAdjJob* d, int njobs, hipStream_t st) {
  if (njobs > 0) hipLaunchKernelGGL(ls_adjoint_kernel, dim3(njobs), dim3(256), 0, st, d);
}
void launch_bilinear(const BilinJob* d, int njobs, int tiles, double* acc, hipStream_t st) {
  if (njobs > 0 && tiles > 0) hipLaunchKernelGGL(bilinear_kernel, dim3(tiles), dim3(256), 0, st, d, njobs, acc);
}

}  // namespace mlh

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
//   hq_update_kernel   every later column Y <- H^H Y = Y - V T^H (V^H Y),
//                      the solve's right-hand sides included, 32 columns per
//                      workgroup, one wavefront per column;
//   hq_backsub_kernel  R X = (Q^H C)[0:c] by back substitution, 32 columns
//                      per workgroup with the tile in LDS.
#include "internal.hpp"

namespace mlh {

__device__ inline double2 hld(const cplx* p) { return *reinterpret_cast<const double2*>(p); }
__device__ inline void hst(cplx* p, double2 v) { *reinterpret_cast<double2*>(p) = v; }

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

// panel rows k..M-1 of columns k..k+15 in LDS (stride 17 against bank conflicts)
__global__ __launch_bounds__(256) void hq_panel_kernel(const HqDesc* __restrict__ descs, int k) {
  const HqDesc& D = descs[blockIdx.x];
  const int c = D.c, M = D.m + c;
  if (k >= c) return;
  const int nb = min(kHqNb, c - k);
  const int L = M - k;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double2 pan[kHqMaxRows][kHqNb + 1];
  __shared__ double red[4];
  __shared__ double2 sh_scale;
  __shared__ double2 tau[kHqNb];
  __shared__ double2 gram[kHqNb][kHqNb + 1];
  __shared__ double2 wcol[kHqNb];
  cplx* A = D.A;
  for (int e = tid; e < L * kHqNb; e += 256) {
    const int r = e % L, j = e / L;
    pan[r][j] = j < nb ? hld(A + (size_t)(k + j) * M + k + r) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    double acc = 0.0;
    for (int r = i + 1 + tid; r < L; r += 256) {
      const double2 x = pan[r][i];
      acc += x.x * x.x + x.y * x.y;
    }
    acc = hwave_sum(acc);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (tid == 0) {
      const double xn2 = red[0] + red[1] + red[2] + red[3];
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
      tau[i] = make_double2(tr, ti);
      sh_scale = make_double2(sr, si);
      pan[i][i] = make_double2(beta, 0.0);
    }
    __syncthreads();
    const double2 sc = sh_scale;
    for (int r = i + 1 + tid; r < L; r += 256) {
      const double2 x = pan[r][i];
      pan[r][i] = make_double2(x.x * sc.x - x.y * sc.y, x.x * sc.y + x.y * sc.x);
    }
    __syncthreads();
    // H_i^H on the panel's later columns: one wavefront per column
    const double2 t = tau[i];
    for (int jj = i + 1 + wave; jj < nb; jj += 4) {
      double wr = 0.0, wi = 0.0;
      for (int r = i + lane; r < L; r += 64) {
        const double2 v = r == i ? make_double2(1.0, 0.0) : pan[r][i];
        const double2 b = pan[r][jj];
        wr += v.x * b.x + v.y * b.y;
        wi += v.x * b.y - v.y * b.x;
      }
      wr = hwave_sum(wr);
      wi = hwave_sum(wi);
      const double tr2 = t.x * wr + t.y * wi, ti2 = t.x * wi - t.y * wr;  // conj(tau) w
      for (int r = i + lane; r < L; r += 64) {
        const double2 v = r == i ? make_double2(1.0, 0.0) : pan[r][i];
        double2 b = pan[r][jj];
        b.x -= v.x * tr2 - v.y * ti2;
        b.y -= v.x * ti2 + v.y * tr2;
        pan[r][jj] = b;
      }
    }
    __syncthreads();
  }
  // Gram matrix G = V^H V (V unit lower trapezoidal) for the T factor
  for (int e = wave; e < nb * nb; e += 4) {
    const int a = e % nb, b = e / nb;
    if (a >= b) continue;  // need G[a][b] for a < b
    double gr = 0.0, gi = 0.0;
    for (int r = b + lane; r < L; r += 64) {
      const double2 va = r == a ? make_double2(1.0, 0.0) : pan[r][a];
      const double2 vb = r == b ? make_double2(1.0, 0.0) : pan[r][b];
      gr += va.x * vb.x + va.y * vb.y;
      gi += va.x * vb.y - va.y * vb.x;
    }
    gr = hwave_sum(gr);
    gi = hwave_sum(gi);
    if (lane == 0) gram[a][b] = make_double2(gr, gi);
  }
  __syncthreads();
  // T: T[i][i] = tau_i ; T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
  __shared__ double2 T[kHqNb][kHqNb + 1];
  for (int e = tid; e < kHqNb * kHqNb; e += 256) T[e % kHqNb][e / kHqNb] = make_double2(0.0, 0.0);
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < nb; ++i) {
      for (int a = 0; a < i; ++a) {
        double2 s = make_double2(0.0, 0.0);
        for (int q = a; q < i; ++q) {
          const double2 x = T[a][q], g = gram[q][i];
          s.x += x.x * g.x - x.y * g.y;
          s.y += x.x * g.y + x.y * g.x;
        }
        wcol[a] = s;
      }
      const double2 ti = tau[i];
      for (int a = 0; a < i; ++a) {
        const double2 s = wcol[a];
        T[a][i] = make_double2(-(ti.x * s.x - ti.y * s.y), -(ti.x * s.y + ti.y * s.x));
      }
      T[i][i] = ti;
    }
  }
  __syncthreads();
  for (int e = tid; e < kHqNb * kHqNb; e += 256) hst(D.T + e, T[e % kHqNb][e / kHqNb]);
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
  const int total = c + D.ncol;
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
  for (int e = tid; e < kHqNb * kHqNb; e += 256) T[e % kHqNb][e / kHqNb] = hld(D.T + e);
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

__global__ __launch_bounds__(256) void hq_backsub_kernel(const HqDesc* __restrict__ descs) {
  const HqDesc& D = descs[blockIdx.y];
  const int c = D.c, M = D.m + c;
  const int col0 = blockIdx.x * kHqCols;
  if (col0 >= D.ncol) return;
  const int nc = min(kHqCols, D.ncol - col0);
  const int tid = threadIdx.x;
  __shared__ double2 z[kHqMaxC][kHqCols + 1];
  __shared__ double2 xk[kHqCols];
  cplx* A = D.A;
  cplx* B = A + (size_t)c * M;  // right-hand sides start after the c columns of S
  for (int e = tid; e < c * kHqCols; e += 256) {
    const int r = e % c, j = e / c;
    z[r][j] = j < nc ? hld(B + (size_t)(col0 + j) * M + r) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int j = tid % kHqCols, rg = tid / kHqCols;  // 8 row groups
  for (int kc = c - 1; kc >= 0; --kc) {
    const cplx* rc = A + (size_t)kc * M;
    if (tid < kHqCols) {
      const double rkk = hld(rc + kc).x;
      const double2 b = z[kc][tid];
      const double2 x = make_double2(b.x / rkk, b.y / rkk);
      xk[tid] = x;
      z[kc][tid] = x;
    }
    __syncthreads();
    const double2 x = xk[j];
    for (int r = rg; r < kc; r += 8) {
      const double2 a = hld(rc + r);
      double2 b = z[r][j];
      b.x -= a.x * x.x - a.y * x.y;
      b.y -= a.x * x.y + a.y * x.x;
      z[r][j] = b;
    }
    __syncthreads();
  }
  for (int e = tid; e < c * kHqCols; e += 256) {
    const int r = e % c, jj = e / c;
    if (jj < nc) hst(B + (size_t)(col0 + jj) * M + r, z[r][jj]);
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
void launch_hq_backsub(const HqDesc* d, int n, int max_ncol, hipStream_t st) {
  const int tiles = (max_ncol + kHqCols - 1) / kHqCols;
  if (n > 0 && tiles > 0) hipLaunchKernelGGL(hq_backsub_kernel, dim3(tiles, n), dim3(256), 0, st, d);
}

}  // namespace mlh

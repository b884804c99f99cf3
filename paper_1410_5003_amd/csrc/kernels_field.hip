// Field evaluation from a solved stack (Sec. 3.3, last paragraph).
//
//  proxy_strength_kernel  c_j = -X_j[0:P, :] [eta_{j-1}; eta_j] for every
//                         layer j (the proxy rows of the layer least-squares
//                         solutions applied to the densities); one workgroup
//                         per layer, one thread per proxy.
//  field_kernel           the scattered field at a tile of up to 256 targets
//                         that lie in one region: inside layer j its
//                         representation eq. (16)-(18) (the near-field
//                         single- and double-layer potentials of the
//                         bounding interfaces over the copies l = -1, 0, 1
//                         with phase alpha^l, eq. (14), plus the proxy
//                         expansion with phi_p = dG/dn_p + i k G, eq. (15));
//                         above U / below D the Rayleigh-Bloch expansion
//                         eq. (7) / (8).  Source nodes are staged through LDS
//                         in chunks shared by the tile's 256 threads; each
//                         thread owns one target and multiplies its sum by
//                         the quasi-periodic phase alpha^m of its cell.
#include "internal.hpp"

namespace mlh {

__global__ __launch_bounds__(256) void proxy_strength_kernel(const ProxyStrengthJob* __restrict__ jobs) {
  const ProxyStrengthJob& J = jobs[blockIdx.x];
  for (int p = threadIdx.x; p < J.P; p += 256) {
    double re = 0.0, im = 0.0;
    for (int part = 0; part < 2; ++part) {
      const cplx* X = J.X + (size_t)(part ? J.n0 : 0) * J.ldX + p;
      const cplx* e = part ? J.eta1 : J.eta0;
      const int n = part ? J.n1 : J.n0;
      for (int c = 0; c < n; ++c) {
        const double2 x = ldc(X + (size_t)c * J.ldX);
        const double2 v = ldc(e + c);
        re += x.x * v.x - x.y * v.y;
        im += x.x * v.y + x.y * v.x;
      }
    }
    stc(J.c + p, -re, -im);
  }
}

// S = (i/4) H0(k r), D = (n'.dv)/(2 pi r^2) (1 + g1m) at separation dv = t - s
__device__ inline void sd_kernels(double k, double r2, double npd, cplx& S, cplx& D) {
  const double r = sqrt(r2);
  cplx h0, gm;
  hankel_pieces(k * r, h0, gm);
  S = {-0.25 * h0.im, 0.25 * h0.re};
  const double f = npd / (2.0 * kPi * r2);
  D = {f * (1.0 + gm.re), f * gm.im};
}

constexpr int kFieldChunk = 256;

__global__ __launch_bounds__(256) void field_kernel(const FieldTile* __restrict__ tiles,
                                                    const FieldRegion* __restrict__ regions,
                                                    const FieldTarget* __restrict__ tgt, double* __restrict__ u,
                                                    int* __restrict__ layer_out, FieldConsts fc) {
  const FieldTile T = tiles[blockIdx.x];
  const FieldRegion& Rg = regions[T.region];
  const int t = T.first + (int)threadIdx.x;
  const bool live = (int)threadIdx.x < T.count;
  FieldTarget me{};
  if (live) me = tgt[t];
  double ur = 0.0, ui = 0.0;
  __shared__ double sh[8][kFieldChunk];
  if (Rg.kind != 0) {
    // Rayleigh-Bloch expansion: sum_n a_n e^{i (kappa_n x +- k_n (y - y_line))}
    const double s = Rg.kind == 1 ? 1.0 : -1.0;
    for (int q = 0; q < fc.nK; ++q) {
      const double kap = fc.kappa0 + 2.0 * kPi * (double)(fc.n0 - fc.K + q) / fc.d;
      const double kk = Rg.k * Rg.k - kap * kap;
      double kr = 0.0, ki = 0.0;  // vertical wavenumber, Re >= 0 and Im >= 0
      if (fabs(kk) > 1e-14 * Rg.k * Rg.k) {
        if (kk > 0)
          kr = sqrt(kk);
        else
          ki = sqrt(-kk);
      }
      const double dy = s * (me.y - Rg.yline);
      const double amp = exp(-ki * dy);
      double sn, cs;
      sincos(kap * me.x + kr * dy, &sn, &cs);
      const double2 a = ldc(Rg.amp + q);
      const double er = amp * cs, ei = amp * sn;
      ur += a.x * er - a.y * ei;
      ui += a.x * ei + a.y * er;
    }
  } else {
    const double k = Rg.k;
    // the bounding interfaces, three copies each
    for (int side = 0; side < 2; ++side) {
      const FieldCurve& C = side ? Rg.below : Rg.above;
      if (C.N == 0) continue;
      const double dyb = C.y0;  // node heights are stored relative to y0
      for (int c0 = 0; c0 < C.N; c0 += kFieldChunk) {
        const int nc = min(kFieldChunk, C.N - c0);
        __syncthreads();
        if ((int)threadIdx.x < nc) {
          const int j = c0 + (int)threadIdx.x;
          sh[0][threadIdx.x] = C.x[j];
          sh[1][threadIdx.x] = C.y[j] + dyb;
          sh[2][threadIdx.x] = C.nx[j];
          sh[3][threadIdx.x] = C.ny[j];
          const double w = C.w[j];
          const double2 tau = ldc(C.eta + j), sig = ldc(C.eta + C.N + j);
          sh[4][threadIdx.x] = w * tau.x;
          sh[5][threadIdx.x] = w * tau.y;
          sh[6][threadIdx.x] = w * sig.x;
          sh[7][threadIdx.x] = w * sig.y;
        }
        __syncthreads();
        if (live) {
          for (int l = 0; l < 3; ++l) {
            double pr = 0.0, pi = 0.0;
            const double shift = (double)(l - 1) * fc.d;
            for (int j = 0; j < nc; ++j) {
              const double dx = me.x - (sh[0][j] + shift), dy = me.y - sh[1][j];
              const double r2 = dx * dx + dy * dy;
              cplx S, D;
              sd_kernels(k, r2, sh[2][j] * dx + sh[3][j] * dy, S, D);
              pr += D.re * sh[4][j] - D.im * sh[5][j] + S.re * sh[6][j] - S.im * sh[7][j];
              pi += D.re * sh[5][j] + D.im * sh[4][j] + S.re * sh[7][j] + S.im * sh[6][j];
            }
            const cplx ph = fc.alpha_pow[l];  // alpha^{l-1}
            ur += ph.re * pr - ph.im * pi;
            ui += ph.re * pi + ph.im * pr;
          }
        }
      }
    }
    // proxy expansion
    for (int c0 = 0; c0 < fc.P; c0 += kFieldChunk) {
      const int nc = min(kFieldChunk, fc.P - c0);
      __syncthreads();
      if ((int)threadIdx.x < nc) {
        const int p = c0 + (int)threadIdx.x;
        sh[0][threadIdx.x] = Rg.px[p];
        sh[1][threadIdx.x] = Rg.py[p] + Rg.centre;
        sh[2][threadIdx.x] = Rg.pnx[p];
        sh[3][threadIdx.x] = Rg.pny[p];
        const double2 c = ldc(Rg.coef + p);
        sh[4][threadIdx.x] = c.x;
        sh[5][threadIdx.x] = c.y;
      }
      __syncthreads();
      if (live) {
        for (int p = 0; p < nc; ++p) {
          const double dx = me.x - sh[0][p], dy = me.y - sh[1][p];
          const double r2 = dx * dx + dy * dy;
          cplx S, D;
          sd_kernels(k, r2, sh[2][p] * dx + sh[3][p] * dy, S, D);
          const double fr = D.re - k * S.im, fi = D.im + k * S.re;  // phi = D + i k S
          ur += fr * sh[4][p] - fi * sh[5][p];
          ui += fr * sh[5][p] + fi * sh[4][p];
        }
      }
    }
  }
  if (live) {
    const double vr = me.ph_re * ur - me.ph_im * ui, vi = me.ph_re * ui + me.ph_im * ur;
    stc(reinterpret_cast<cplx*>(u) + me.idx, vr, vi);
    if (layer_out) layer_out[me.idx] = Rg.label;
  }
}

void launch_proxy_strength(const ProxyStrengthJob* d_jobs, int njobs, hipStream_t st) {
  if (njobs > 0) hipLaunchKernelGGL(proxy_strength_kernel, dim3(njobs), dim3(256), 0, st, d_jobs);
}

void launch_field(const FieldTile* d_tiles, int ntiles, const FieldRegion* d_regions, const FieldTarget* d_tgt,
                  double* u, int* layer_out, const FieldConsts& fc, hipStream_t st) {
  for (int t0 = 0; t0 < ntiles; t0 += kMaxLaunchBlocks)
    hipLaunchKernelGGL(field_kernel, dim3(std::min(kMaxLaunchBlocks, ntiles - t0)), dim3(256), 0, st,
                       d_tiles + t0, d_regions, d_tgt, u, layer_out, fc);
}

}  // namespace mlh

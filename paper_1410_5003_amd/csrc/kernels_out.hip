// Output staging of the solve.
//
//  gather_eta_kernel  copies the densities eta_i (Sec. 3.3) of every angle of
//                     a batch from the per-system workspace, where interface
//                     i holds an n_i x r column block, into one row of
//                     N_den = sum_i n_i entries per angle (interfaces in
//                     order, [tau_i; sigma_i] each).

#include "internal.hpp"

namespace mlh {

__global__ __launch_bounds__(256) void gather_eta_kernel(const EtaSeg* __restrict__ seg,
                                                         const EtaDst* __restrict__ dst) {
  const EtaSeg S = seg[blockIdx.y];
  const EtaDst D = dst[blockIdx.z];
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= S.n) return;
  const cplx* src = reinterpret_cast<const cplx*>(D.sys_base + S.src_off) + (size_t)D.col * S.n + r;
  const double2 v = ldc(src);
  stc(D.dst + S.dst_off + r, v.x, v.y);
}

void launch_gather_eta(const EtaSeg* d_seg, int nseg, int max_n, const EtaDst* d_dst, int ndst, hipStream_t st) {
  if (nseg <= 0 || ndst <= 0 || max_n <= 0) return;
  dim3 grid((max_n + 255) / 256, nseg, ndst);
  hipLaunchKernelGGL(gather_eta_kernel, grid, dim3(256), 0, st, d_seg, d_dst);
}

}  // namespace mlh

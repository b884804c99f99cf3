// Output staging of the solve, and the fixed workspace of the
// allocation-free solve.
//
//  gather_eta_kernel  copies the densities eta_i (Sec. 3.3) of every angle of
//                     a batch from the per-system workspace, where interface
//                     i holds an n_i x r column block, into one row of
//                     N_den = sum_i n_i entries per angle (interfaces in
//                     order, [tau_i; sigma_i] each).
//  scratch            kScratchBytes of device memory per GPU, reserved when
//                     the library's code object is loaded on that GPU and
//                     held until the process ends.  Host code never uses the
//                     array's name as an address: scratch_address() looks up
//                     each device's own copy once (hipGetSymbolAddress) and
//                     every launch and copy takes that pointer.

#include <mutex>
#include <vector>

#include "internal.hpp"

namespace mlh {

static __device__ __align__(256) char scratch[kScratchBytes];

hipError_t scratch_address(int device, char** ptr) {
  static std::mutex mu;
  static std::vector<char*> addr;  // per device; null until looked up
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<char*>(p);
  }
  *ptr = addr[device];
  return hipSuccess;
}

__global__ __launch_bounds__(256) void gather_eta_kernel(const EtaSeg* __restrict__ seg,
                                                         const EtaDst* __restrict__ dst) {
  const EtaDst D = dst[blockIdx.z];
  if ((int)blockIdx.y >= D.nseg) return;
  const EtaSeg S = seg[D.seg0 + blockIdx.y];
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= S.n) return;
  const cplx* src = reinterpret_cast<const cplx*>(D.sys_base + S.src_off) + (size_t)D.col * S.n + r;
  const double2 v = ldc(src);
  stc(D.dst + S.dst_off + r, v.x, v.y);
}

void launch_gather_eta(const EtaSeg* d_seg, int max_seg, int max_n, const EtaDst* d_dst, int ndst, hipStream_t st) {
  if (max_seg <= 0 || ndst <= 0 || max_n <= 0) return;
  dim3 grid((max_n + 255) / 256, max_seg, ndst);
  hipLaunchKernelGGL(gather_eta_kernel, grid, dim3(256), 0, st, d_seg, d_dst);
}

}  // namespace mlh

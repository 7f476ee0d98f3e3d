// Host-to-device upload of launch descriptors by a copy kernel that reads the
// pinned staging buffer directly (it is mapped into the device's address
// space).  Unlike an asynchronous copy command, the kernel is ordered on its
// stream like any launch: a stream that waits on another stream's event keeps
// queueing without the host waiting for that event.
#include "kernels.hpp"

namespace symhss {

__global__ __launch_bounds__(256) void k_upload(uint4* __restrict__ dst, const uint4* __restrict__ src, long n16) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n16; e += (long)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

void launch_upload(hipStream_t st, void* dst, const void* src_pinned, size_t bytes) {
  // bytes is a multiple of 16 and both pointers 16-byte aligned (staging
  // chunks hand out 256-byte aligned slices)
  const long n16 = (long)(bytes / 16);
  if (n16 <= 0) return;
  const int grid = (int)std::min<long>(cdiv_int(n16, 256), 256);
  hipLaunchKernelGGL(k_upload, dim3(grid), dim3(256), 0, st, static_cast<uint4*>(dst),
                     static_cast<const uint4*>(src_pinned), n16);
  HIPCHK(hipGetLastError());
}

// na arrays of n doubles stored back to back in pinned staging memory, array
// a copied to dst + a ld (one launch for the parts of a strided table)
__global__ __launch_bounds__(256) void k_upload_split(double* __restrict__ dst, long ld,
                                                      const double* __restrict__ src, long n, int na) {
  const long tot = n * na;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const long a = e / n, i = e - a * n;
    dst[a * ld + i] = src[e];
  }
}

void launch_upload_split(hipStream_t st, double* dst, size_t ld, const double* src_pinned, size_t n, int na) {
  const long tot = (long)n * na;
  if (tot <= 0) return;
  const int grid = (int)std::min<long>(cdiv_int(tot, 256), 256);
  hipLaunchKernelGGL(k_upload_split, dim3(grid), dim3(256), 0, st, dst, (long)ld, src_pinned, (long)n, na);
  HIPCHK(hipGetLastError());
}

}  // namespace symhss

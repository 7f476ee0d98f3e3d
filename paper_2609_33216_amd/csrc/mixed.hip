// Precision conversions and vector kernels of the mixed-precision solve:
// FP64 blocks rounded to FP32 for the factorisation, and the refinement
// steps x += d, r = b - A x and column norms in FP64.
#include "kernels.hpp"

namespace symhss {

__global__ void k_convert_batched(const ConvDesc* __restrict__ descs) {
  const ConvDesc D = descs[blockIdx.y];
  const long total = (long)D.rows * D.cols;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e / D.rows), i = (int)(e - (long)c * D.rows);
    const cplx v = D.src[i + (long)D.lds * c];
    D.dst[i + (long)D.ldd * c] = cplxf{(float)v.re, (float)v.im};
  }
}

// FP32 blocks placed in an FP64 matrix (the dense top-level system's diagonal
// blocks, factored in FP64)
__global__ void k_scatter2_widen(const Scatter2WideDesc* __restrict__ descs) {
  const Scatter2WideDesc S = descs[blockIdx.y];
  const int total = S.m * S.n;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int i = e % S.m, j = e / S.m;
    const cplxf v = S.src[i + (long)S.lds * j];
    S.dst[S.rmap[i] + (long)S.ldd * S.cmap[j]] = cplx{(double)v.re, (double)v.im};
  }
}

// y = (double) x
__global__ void k_widen_vec(const cplxf* __restrict__ x, cplx* __restrict__ y, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    y[e] = cplx{(double)x[e].re, (double)x[e].im};
}

// y = (float) x
__global__ void k_round_vec(const cplx* __restrict__ x, cplxf* __restrict__ y, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    y[e] = cplxf{(float)x[e].re, (float)x[e].im};
}

// x += d (d in FP32)
__global__ void k_add_vec(cplx* __restrict__ x, const cplxf* __restrict__ d, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    x[e].re += (double)d[e].re;
    x[e].im += (double)d[e].im;
  }
}

// r = b - y
__global__ void k_sub_vec(const cplx* __restrict__ b, const cplx* __restrict__ y, cplx* __restrict__ r, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    r[e] = b[e] - y[e];
}

// out[c] = sum_i |v[i + ld c]|^2 in two stages with a fixed summation order:
// kNormParts workgroups per column each sum a contiguous part into
// part[c kNormParts + p], then one workgroup per column adds the parts.
__global__ __launch_bounds__(256) void k_col_norm2_parts(const cplx* __restrict__ v, long n, long ld,
                                                         double* __restrict__ part) {
  __shared__ double red[256];
  const cplx* col = v + ld * blockIdx.y;
  const long chunk = (n + kNormParts - 1) / kNormParts;
  const long i0 = chunk * blockIdx.x, i1 = i0 + chunk < n ? i0 + chunk : n;
  double s = 0.0;
  for (long i = i0 + threadIdx.x; i < i1; i += blockDim.x) s += abs2(col[i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long)kNormParts * blockIdx.y + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kNormParts) void k_col_norm2_sum(const double* __restrict__ part,
                                                              double* __restrict__ out) {
  __shared__ double red[kNormParts];
  red[threadIdx.x] = part[(long)kNormParts * blockIdx.x + threadIdx.x];
  __syncthreads();
  for (int w = kNormParts / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

static int grid_for(long n) { return (int)std::min<long>(std::max<long>(cdiv_int(n, 256), 1), 8192); }

void launch_convert_batched(hipStream_t st, const ConvDesc* d, int count, long maxelems) {
  if (count <= 0 || maxelems <= 0) return;
  hipLaunchKernelGGL(k_convert_batched, dim3(grid_for(maxelems) < 1024 ? grid_for(maxelems) : 1024, count),
                     dim3(256), 0, st, d);
  HIPCHK(hipGetLastError());
}

void launch_scatter2_widen(hipStream_t st, const Scatter2WideDesc* d, int count, long maxelems) {
  if (count <= 0 || maxelems <= 0) return;
  hipLaunchKernelGGL(k_scatter2_widen, dim3(grid_for(maxelems) < 1024 ? grid_for(maxelems) : 1024, count),
                     dim3(256), 0, st, d);
  HIPCHK(hipGetLastError());
}

void launch_widen_vec(hipStream_t st, const cplxf* x, cplx* y, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_widen_vec, dim3(grid_for(n)), dim3(256), 0, st, x, y, n);
  HIPCHK(hipGetLastError());
}

void launch_round_vec(hipStream_t st, const cplx* x, cplxf* y, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_round_vec, dim3(grid_for(n)), dim3(256), 0, st, x, y, n);
  HIPCHK(hipGetLastError());
}

void launch_add_vec(hipStream_t st, cplx* x, const cplxf* d, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_add_vec, dim3(grid_for(n)), dim3(256), 0, st, x, d, n);
  HIPCHK(hipGetLastError());
}

void launch_sub_vec(hipStream_t st, const cplx* b, const cplx* y, cplx* r, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sub_vec, dim3(grid_for(n)), dim3(256), 0, st, b, y, r, n);
  HIPCHK(hipGetLastError());
}

void launch_col_norm2(hipStream_t st, const cplx* v, long n, long ld, int ncols, double* out, double* work) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_col_norm2_parts, dim3(kNormParts, ncols), dim3(256), 0, st, v, n, ld, work);
  hipLaunchKernelGGL(k_col_norm2_sum, dim3(ncols), dim3(kNormParts), 0, st, work, out);
  HIPCHK(hipGetLastError());
}

}  // namespace symhss

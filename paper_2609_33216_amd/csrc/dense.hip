// Batched dense complex FP64 linear algebra for the compressed equations of
// paper Section 4.2: LU with partial pivoting of each diagonal block with its
// right-hand sides appended (so that X = D^{-1} L falls out of the same
// factorisation), the GEMMs R X, A~ R g, X z, triangular solves, and the
// gathers that assemble a parent's diagonal block from its children.
//
// All matrices are column-major.  A workgroup of 256 threads computes a
// 64 x 64 output tile of a GEMM as 16 x 16 threads with 4 x 4 accumulators
// each, staging 16-deep slices of both operands in LDS.
#include "kernels.hpp"

namespace symhss {

constexpr int kTile = 64;
constexpr int kKC = 16;
constexpr int kNB = 32;  // LU panel width





// One 64 x 64 tile of C = beta C + alpha A B computed by the workgroup.
__device__ void tile_gemm(int m, int n, int k, const cplx* __restrict__ A, long lda, const cplx* __restrict__ B,
                          long ldb, cplx* __restrict__ C, long ldc, double alpha, double beta, int r0, int c0,
                          cplx* lds) {
  cplx* As = lds;                  // [kKC][kTile]
  cplx* Bs = lds + kKC * kTile;    // [kKC][kTile]
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  cplx acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = mk(0, 0);
  for (int k0 = 0; k0 < k; k0 += kKC) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int row = e & 63, kk = e >> 6;
      const int gr = r0 + row, gk = k0 + kk;
      As[kk * kTile + row] = (gr < m && gk < k) ? A[gr + lda * gk] : mk(0, 0);
      const int kb = e & 15, col = e >> 4;
      const int gk2 = k0 + kb, gc = c0 + col;
      Bs[kb * kTile + col] = (gk2 < k && gc < n) ? B[gk2 + ldb * gc] : mk(0, 0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kKC; ++kk) {
      cplx a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk * kTile + tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk * kTile + ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) fma_acc(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int gc = c0 + ty + 16 * j;
    if (gc >= n) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int gr = r0 + tx + 16 * i;
      if (gr >= m) continue;
      cplx* p = C + gr + ldc * gc;
      cplx v = mk(alpha * acc[i][j].re, alpha * acc[i][j].im);
      if (beta != 0.0) v = v + beta * (*p);
      *p = v;
    }
  }
}

// Whole GEMM by one workgroup (loops over its tiles).
__device__ void wg_gemm(int m, int n, int k, const cplx* A, long lda, const cplx* B, long ldb, cplx* C, long ldc,
                        double alpha, double beta, cplx* lds) {
  if (m <= 0 || n <= 0) return;
  for (int c0 = 0; c0 < n; c0 += kTile)
    for (int r0 = 0; r0 < m; r0 += kTile) tile_gemm(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, r0, c0, lds);
}

__global__ __launch_bounds__(256) void k_gemm_batched(const GemmDesc* __restrict__ descs) {
  __shared__ cplx lds[2 * kKC * kTile];
  const GemmDesc G = descs[blockIdx.z];
  const int r0 = blockIdx.x * kTile, c0 = blockIdx.y * kTile;
  if (r0 >= G.m || c0 >= G.n) return;
  tile_gemm(G.m, G.n, G.k, G.A, G.lda, G.B, G.ldb, G.C, G.ldc, G.alpha, G.beta, r0, c0, lds);
}

__device__ inline void wg_argmax_abs(const cplx* col, int lo, int hi, int& piv, double& pval, double* sval,
                                     int* sidx) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double best = -1.0;
  int bi = lo;
  for (int i = lo + tid; i < hi; i += 256) {
    const double v = abs2(col[i]);
    if (v > best) { best = v; bi = i; }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  if (lane == 0) { sval[wave] = best; sidx[wave] = bi; }
  __syncthreads();
  if (tid == 0) {
    double b = sval[0];
    int ix = sidx[0];
    for (int w = 1; w < 4; ++w)
      if (sval[w] > b || (sval[w] == b && sidx[w] < ix)) { b = sval[w]; ix = sidx[w]; }
    sval[4] = b;
    sidx[4] = ix;
  }
  __syncthreads();
  piv = sidx[4];
  pval = sval[4];
  __syncthreads();
}

// Right-looking blocked LU with partial pivoting of A[0:n, 0:n] with row
// interchanges applied to all ncol columns, then backward substitution on
// the appended columns: on exit A[0:n, n:ncol] = D^{-1} (original appended
// columns).  One workgroup per matrix.
__global__ __launch_bounds__(256) void k_lu_fused(const LuDesc* __restrict__ descs) {
  __shared__ cplx lds[2 * kKC * kTile];
  __shared__ double sval[5];
  __shared__ int sidx[5];
  const LuDesc D = descs[blockIdx.x];
  const int n = D.n, nc = D.ncol;
  const long lda = D.lda;
  cplx* A = D.A;
  const int tid = threadIdx.x;
  for (int j = 0; j < n; j += kNB) {
    const int jb = min(kNB, n - j);
    for (int jj = j; jj < j + jb; ++jj) {
      int p;
      double pv;
      wg_argmax_abs(A + lda * jj, jj, n, p, pv, sval, sidx);
      if (tid == 0) {
        D.ipiv[jj] = p;
        if (pv == 0.0 && *D.info == 0) *D.info = jj + 1;
      }
      if (p != jj) {
        for (int c = tid; c < nc; c += 256) {
          const cplx t = A[jj + lda * c];
          A[jj + lda * c] = A[p + lda * c];
          A[p + lda * c] = t;
        }
      }
      __syncthreads();
      const cplx pivv = A[jj + lda * jj];
      const cplx inv = (pv == 0.0) ? mk(0, 0) : cdiv(mk(1, 0), pivv);
      for (int i = jj + 1 + tid; i < n; i += 256) {
        const cplx l = A[i + lda * jj] * inv;
        A[i + lda * jj] = l;
        for (int c = jj + 1; c < j + jb; ++c) {
          const cplx u = A[jj + lda * c];
          cplx a = A[i + lda * c];
          a.re -= l.re * u.re - l.im * u.im;
          a.im -= l.re * u.im + l.im * u.re;
          A[i + lda * c] = a;
        }
      }
      __syncthreads();
    }
    // U12 = L11^{-1} A12 (unit lower triangular L11)
    for (int c = j + jb + tid; c < nc; c += 256) {
      for (int r = 1; r < jb; ++r) {
        cplx s = A[j + r + lda * c];
        for (int l = 0; l < r; ++l) {
          const cplx L = A[j + r + lda * (j + l)];
          const cplx x = A[j + l + lda * c];
          s.re -= L.re * x.re - L.im * x.im;
          s.im -= L.re * x.im + L.im * x.re;
        }
        A[j + r + lda * c] = s;
      }
    }
    __syncthreads();
    wg_gemm(n - j - jb, nc - j - jb, jb, A + (j + jb) + lda * j, lda, A + j + lda * (j + jb), lda,
            A + (j + jb) + lda * (j + jb), lda, -1.0, 1.0, lds);
    __syncthreads();
  }
  if (nc == n) return;
  // backward substitution with U on the appended columns, blocked from the bottom
  const int nb0 = ((n - 1) / kNB) * kNB;
  for (int j = nb0; j >= 0; j -= kNB) {
    const int jb = min(kNB, n - j);
    for (int c = n + tid; c < nc; c += 256) {
      for (int r = jb - 1; r >= 0; --r) {
        cplx s = A[j + r + lda * c];
        for (int l = r + 1; l < jb; ++l) {
          const cplx U = A[j + r + lda * (j + l)];
          const cplx x = A[j + l + lda * c];
          s.re -= U.re * x.re - U.im * x.im;
          s.im -= U.re * x.im + U.im * x.re;
        }
        A[j + r + lda * c] = cdiv(s, A[j + r + lda * (j + r)]);
      }
    }
    __syncthreads();
    wg_gemm(j, nc - n, jb, A + lda * j, lda, A + j + lda * n, lda, A + lda * n, lda, -1.0, 1.0, lds);
    __syncthreads();
  }
}


__global__ __launch_bounds__(256) void k_lu_solve(const SolveDesc* __restrict__ descs) {
  const SolveDesc S = descs[blockIdx.x];
  const int n = S.n;
  const long lda = S.lda, ldb = S.ldb;
  const int tid = threadIdx.x;
  // row interchanges (sequential in their order), one thread per rhs column
  for (int c = tid; c < S.nrhs; c += 256) {
    cplx* b = S.B + ldb * c;
    for (int i = 0; i < n; ++i) {
      const int p = S.ipiv[i];
      if (p != i) {
        const cplx t = b[i];
        b[i] = b[p];
        b[p] = t;
      }
    }
  }
  __syncthreads();
  for (int c = 0; c < S.nrhs; ++c) {
    cplx* b = S.B + ldb * c;
    for (int j = 0; j < n; ++j) {
      const cplx x = b[j];
      for (int i = j + 1 + tid; i < n; i += 256) {
        const cplx L = S.LU[i + lda * j];
        b[i].re -= L.re * x.re - L.im * x.im;
        b[i].im -= L.re * x.im + L.im * x.re;
      }
      __syncthreads();
    }
    for (int j = n - 1; j >= 0; --j) {
      if (tid == 0) b[j] = cdiv(b[j], S.LU[j + lda * j]);
      __syncthreads();
      const cplx x = b[j];
      for (int i = tid; i < j; i += 256) {
        const cplx U = S.LU[i + lda * j];
        b[i].re -= U.re * x.re - U.im * x.im;
        b[i].im -= U.re * x.im + U.im * x.re;
      }
      __syncthreads();
    }
  }
}

__global__ void k_copy_batched(const CopyDesc* __restrict__ descs) {
  const CopyDesc C = descs[blockIdx.y];
  const int total = C.rows * C.cols;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int i = e % C.rows, c = e / C.rows;
    const int si = C.smap ? C.smap[i] : i;
    const int di = C.dmap ? C.dmap[i] : i;
    C.dst[di + (long)C.ldd * c] = C.src[si + (long)C.lds * c];
  }
}

__global__ void k_scatter2_batched(const Scatter2Desc* __restrict__ descs) {
  const Scatter2Desc S = descs[blockIdx.y];
  const int total = S.m * S.n;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int i = e % S.m, j = e / S.m;
    S.dst[S.rmap[i] + (long)S.ldd * S.cmap[j]] = S.src[i + (long)S.lds * j];
  }
}

__global__ void k_zero(cplx* p, long count) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x)
    p[e] = mk(0, 0);
}

// identity block appended to each matrix: A[i, n + i] = 1 (the rest zeroed by k_zero)
__global__ void k_set_identity(const LuDesc* __restrict__ descs) {
  const LuDesc D = descs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D.n && D.n + i < D.ncol) D.A[i + (long)D.lda * (D.n + i)] = mk(1, 0);
}

void launch_lu_fused(hipStream_t st, const LuDesc* d, int count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_lu_fused, dim3(count), dim3(256), 0, st, d);
  HIPCHK(hipGetLastError());
}

void launch_gemm_batched(hipStream_t st, const GemmDesc* d, int count, int mmax, int nmax) {
  if (count <= 0 || mmax <= 0 || nmax <= 0) return;
  hipLaunchKernelGGL(k_gemm_batched, dim3(cdiv_int(mmax, kTile), cdiv_int(nmax, kTile), count), dim3(256), 0, st,
                     d);
  HIPCHK(hipGetLastError());
}

void launch_lu_solve(hipStream_t st, const SolveDesc* d, int count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_lu_solve, dim3(count), dim3(256), 0, st, d);
  HIPCHK(hipGetLastError());
}

void launch_copy_batched(hipStream_t st, const CopyDesc* d, int count, long maxelems) {
  if (count <= 0 || maxelems <= 0) return;
  const int gx = (int)std::min<long>(cdiv_int(maxelems, 256), 1024);
  hipLaunchKernelGGL(k_copy_batched, dim3(gx, count), dim3(256), 0, st, d);
  HIPCHK(hipGetLastError());
}

void launch_scatter2_batched(hipStream_t st, const Scatter2Desc* d, int count, long maxelems) {
  if (count <= 0 || maxelems <= 0) return;
  const int gx = (int)std::min<long>(cdiv_int(maxelems, 256), 1024);
  hipLaunchKernelGGL(k_scatter2_batched, dim3(gx, count), dim3(256), 0, st, d);
  HIPCHK(hipGetLastError());
}

void launch_zero(hipStream_t st, cplx* p, long count) {
  if (count <= 0) return;
  const int g = (int)std::min<long>(cdiv_int(count, 256), 8192);
  hipLaunchKernelGGL(k_zero, dim3(g), dim3(256), 0, st, p, count);
  HIPCHK(hipGetLastError());
}

void launch_set_identity(hipStream_t st, const LuDesc* d, int count, int nmax) {
  if (count <= 0 || nmax <= 0) return;
  hipLaunchKernelGGL(k_set_identity, dim3(cdiv_int(nmax, 256), count), dim3(256), 0, st, d);
  HIPCHK(hipGetLastError());
}

}  // namespace symhss

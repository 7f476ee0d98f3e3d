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


// Factor the panel A[j:n, j:j+jb] with partial pivoting; row interchanges are
// applied inside the panel only (the caller applies them to the other columns).
__device__ void wg_lu_panel(const LuDesc& D, int j, int jb, double* sval, int* sidx) {
  __shared__ cplx urow[kNB];
  const int n = D.n;
  const long lda = D.lda;
  cplx* A = D.A;
  const int tid = threadIdx.x;
  for (int jj = j; jj < j + jb; ++jj) {
    int p;
    double pv;
    wg_argmax_abs(A + lda * jj, jj, n, p, pv, sval, sidx);
    if (tid == 0) {
      D.ipiv[jj] = p;
      if (pv == 0.0 && *D.info == 0) *D.info = jj + 1;
    }
    if (tid < jb) {
      const int c = j + tid;
      cplx t = A[jj + lda * c];
      if (p != jj) {
        const cplx o = A[p + lda * c];
        A[jj + lda * c] = o;
        A[p + lda * c] = t;
        t = o;
      }
      urow[tid] = t;  // pivot row of the panel after the interchange
    }
    __syncthreads();
    const cplx pivv = urow[jj - j];
    const cplx inv = (pv == 0.0) ? mk(0, 0) : cdiv(mk(1, 0), pivv);
    const int c0 = jj + 1 - j;  // first panel column to update (local index)
    for (int i = jj + 1 + tid; i < n; i += 256) {
      const cplx l = A[i + lda * jj] * inv;
      A[i + lda * jj] = l;
      cplx* row = A + i;
      // eight independent loads in flight per chunk
      for (int cb = c0; cb < jb; cb += 8) {
        cplx a[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (cb + q < jb) a[q] = row[lda * (j + cb + q)];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (cb + q < jb) {
            const cplx u = urow[cb + q];
            a[q].re -= l.re * u.re - l.im * u.im;
            a[q].im -= l.re * u.im + l.im * u.re;
            row[lda * (j + cb + q)] = a[q];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Row interchanges of panel [j, j+jb) applied to one column outside the panel.
__device__ inline void apply_swaps(const LuDesc& D, int j, int jb, int c) {
  const long lda = D.lda;
  cplx* col = D.A + lda * c;
  for (int jj = j; jj < j + jb; ++jj) {
    const int p = D.ipiv[jj];
    if (p != jj) {
      const cplx t = col[jj];
      col[jj] = col[p];
      col[p] = t;
    }
  }
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
    wg_lu_panel(D, j, jb, sval, sidx);
    for (int c = tid; c < nc - jb; c += 256) apply_swaps(D, j, jb, c < j ? c : c + jb);
    __syncthreads();
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


// Forward (unit L) and backward (U) substitution in 64-row blocks: wavefront
// 0 solves the diagonal block with lane shuffles, then all threads update the
// remaining rows; two barriers per block.
__device__ inline cplx shfl_c(cplx v, int src) {
  return mk(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}

__global__ __launch_bounds__(256) void k_lu_solve(const SolveDesc* __restrict__ descs) {
  __shared__ cplx Dg[64 * 64];
  __shared__ cplx xs[64];
  const SolveDesc S = descs[blockIdx.x];
  const int n = S.n;
  const long lda = S.lda, ldb = S.ldb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
    for (int j0 = 0; j0 < n; j0 += 64) {
      const int jb = min(64, n - j0);
      for (int q = tid; q < 64 * 64; q += 256) {
        const int r = q & 63, cc = q >> 6;
        Dg[q] = (r < jb && cc < jb) ? S.LU[j0 + r + lda * (j0 + cc)] : mk(0, 0);
      }
      __syncthreads();
      if (wave == 0) {
        cplx x = lane < jb ? b[j0 + lane] : mk(0, 0);
        for (int l = 0; l < jb; ++l) {
          const cplx xl = shfl_c(x, l);
          if (lane > l && lane < jb) {
            const cplx L = Dg[lane + 64 * l];
            x.re -= L.re * xl.re - L.im * xl.im;
            x.im -= L.re * xl.im + L.im * xl.re;
          }
        }
        if (lane < jb) b[j0 + lane] = x;
      }
      __syncthreads();
      for (int q = tid; q < jb; q += 256) xs[q] = b[j0 + q];
      __syncthreads();
      for (int i = j0 + jb + tid; i < n; i += 256) {
        cplx s = b[i];
        const cplx* Li = S.LU + i + lda * j0;
#pragma unroll 8
        for (int l = 0; l < jb; ++l) {
          const cplx L = Li[lda * l];
          const cplx x = xs[l];
          s.re -= L.re * x.re - L.im * x.im;
          s.im -= L.re * x.im + L.im * x.re;
        }
        b[i] = s;
      }
      __syncthreads();
    }
    const int nb0 = n > 0 ? ((n - 1) / 64) * 64 : -1;
    for (int j0 = nb0; j0 >= 0; j0 -= 64) {
      const int jb = min(64, n - j0);
      for (int q = tid; q < 64 * 64; q += 256) {
        const int r = q & 63, cc = q >> 6;
        Dg[q] = (r < jb && cc < jb) ? S.LU[j0 + r + lda * (j0 + cc)] : mk(1, 0);
      }
      __syncthreads();
      if (wave == 0) {
        cplx x = lane < jb ? b[j0 + lane] : mk(0, 0);
        for (int l = jb - 1; l >= 0; --l) {
          if (lane == l) x = cdiv(x, Dg[l + 64 * l]);
          const cplx xl = shfl_c(x, l);
          if (lane < l) {
            const cplx U = Dg[lane + 64 * l];
            x.re -= U.re * xl.re - U.im * xl.im;
            x.im -= U.re * xl.im + U.im * xl.re;
          }
        }
        if (lane < jb) b[j0 + lane] = x;
      }
      __syncthreads();
      for (int q = tid; q < jb; q += 256) xs[q] = b[j0 + q];
      __syncthreads();
      for (int i = tid; i < j0; i += 256) {
        cplx s = b[i];
        const cplx* Ui = S.LU + i + lda * j0;
#pragma unroll 8
        for (int l = 0; l < jb; ++l) {
          const cplx U = Ui[lda * l];
          const cplx x = xs[l];
          s.re -= U.re * x.re - U.im * x.im;
          s.im -= U.re * x.im + U.im * x.re;
        }
        b[i] = s;
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


// ---------------------------------------------------------------------------
// Multi-workgroup blocked LU for batches of few, large matrices: the host
// loops over panels; each panel step is three launches (panel factorisation
// by one workgroup per matrix, row-block triangular solve and trailing GEMM
// spread over many workgroups).  Same arithmetic as k_lu_fused.

__global__ __launch_bounds__(256) void k_lu_panel(const LuDesc* __restrict__ descs, int j) {
  __shared__ double sval[5];
  __shared__ int sidx[5];
  const LuDesc D = descs[blockIdx.x];
  if (j >= D.n) return;
  wg_lu_panel(D, j, min(kNB, D.n - j), sval, sidx);
}

// Columns outside panel [j, j+jb), 64 per workgroup: apply the panel's row
// interchanges; for columns right of the panel also U12 = L11^{-1} A12, as a
// product with the explicit inverse of the unit lower triangular L11 (formed
// in LDS by one wavefront, one column of the inverse per lane).
__global__ __launch_bounds__(256) void k_lu_swap_trsm(const LuDesc* __restrict__ descs, int j) {
  __shared__ cplx Linv[kNB * kNB];
  __shared__ cplx Bs[kNB * 64];
  const LuDesc D = descs[blockIdx.y];
  const int n = D.n, nc = D.ncol;
  if (j >= n) return;
  const long lda = D.lda;
  const int jb = min(kNB, n - j);
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * 64;
  if (e0 >= nc - jb) return;
  if (tid < 64) {
    const int e = e0 + tid;
    if (e < nc - jb) apply_swaps(D, j, jb, e < j ? e : e + jb);
  }
  // columns of this block right of the panel: e >= j
  if (e0 + 63 < j) return;
  if (tid < 64) {
    // column tid of L11^{-1}: solve L11 x = e_tid by forward substitution
    if (tid < kNB) {
      for (int r = 0; r < kNB; ++r) Linv[r + kNB * tid] = mk(r == tid ? 1.0 : 0.0, 0.0);
      if (tid < jb) {
        for (int r = tid + 1; r < jb; ++r) {
          cplx s = mk(0, 0);
          for (int l = tid; l < r; ++l) {
            const cplx L = D.A[j + r + lda * (j + l)];
            const cplx x = Linv[l + kNB * tid];
            s.re -= L.re * x.re - L.im * x.im;
            s.im -= L.re * x.im + L.im * x.re;
          }
          Linv[r + kNB * tid] = s;
        }
      }
    }
  }
  __syncthreads();  // swaps of this block's columns and Linv are complete
  for (int q = tid; q < kNB * 64; q += 256) {
    const int r = q % kNB, cc = q / kNB;
    const int e = e0 + cc;
    const bool ok = e >= j && e < nc - jb && r < jb;
    Bs[q] = ok ? D.A[j + r + lda * (e + jb)] : mk(0, 0);
  }
  __syncthreads();
  for (int q = tid; q < kNB * 64; q += 256) {
    const int r = q % kNB, cc = q / kNB;
    const int e = e0 + cc;
    if (!(e >= j && e < nc - jb && r < jb)) continue;
    cplx acc = mk(0, 0);
    for (int l = 0; l <= r; ++l) fma_acc(acc, Linv[r + kNB * l], Bs[l + kNB * cc]);
    D.A[j + r + lda * (e + jb)] = acc;
  }
}

// A22 -= L21 U12, one 64 x 64 tile per workgroup.
__global__ __launch_bounds__(256) void k_lu_update(const LuDesc* __restrict__ descs, int j) {
  __shared__ cplx lds[2 * kKC * kTile];
  const LuDesc D = descs[blockIdx.z];
  const int n = D.n, nc = D.ncol;
  if (j >= n) return;
  const int jb = min(kNB, n - j);
  const int m = n - j - jb, ncols = nc - j - jb;
  const int r0 = blockIdx.x * kTile, c0 = blockIdx.y * kTile;
  if (r0 >= m || c0 >= ncols) return;
  const long lda = D.lda;
  cplx* A = D.A;
  tile_gemm(m, ncols, jb, A + (j + jb) + lda * j, lda, A + j + lda * (j + jb), lda, A + (j + jb) + lda * (j + jb),
            lda, -1.0, 1.0, r0, c0, lds);
}

// Backward substitution on the appended columns, block row [j, j + jb):
// X_j = U_jj^{-1} B_j; then B[0:j] -= U[0:j, j:j+jb] X_j (k_lu_backupdate).
__global__ __launch_bounds__(256) void k_lu_trsm_upper(const LuDesc* __restrict__ descs, int j) {
  __shared__ cplx U[kNB * kNB];
  const LuDesc D = descs[blockIdx.y];
  const int n = D.n, nc = D.ncol;
  if (j >= n || nc == n) return;
  const long lda = D.lda;
  const int jb = min(kNB, n - j);
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int r = e % kNB, c = e / kNB;
    U[e] = (r < jb && c < jb) ? D.A[j + r + lda * (j + c)] : mk(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int c = n + blockIdx.x * 256 + threadIdx.x;
  if (c >= nc) return;
  cplx x[kNB];
#pragma unroll
  for (int r = 0; r < kNB; ++r) x[r] = (r < jb) ? D.A[j + r + lda * c] : mk(0, 0);
#pragma unroll
  for (int r = kNB - 1; r >= 0; --r) {
    cplx s = x[r];
#pragma unroll
    for (int l = r + 1; l < kNB; ++l) {
      const cplx u = U[r + kNB * l];
      s.re -= u.re * x[l].re - u.im * x[l].im;
      s.im -= u.re * x[l].im + u.im * x[l].re;
    }
    x[r] = cdiv(s, U[r + kNB * r]);
  }
#pragma unroll
  for (int r = 0; r < kNB; ++r)
    if (r < jb) D.A[j + r + lda * c] = x[r];
}

__global__ __launch_bounds__(256) void k_lu_backupdate(const LuDesc* __restrict__ descs, int j) {
  __shared__ cplx lds[2 * kKC * kTile];
  const LuDesc D = descs[blockIdx.z];
  const int n = D.n, nc = D.ncol;
  if (j >= n || nc == n) return;
  const int jb = min(kNB, n - j);
  const int m = j, ncols = nc - n;
  const int r0 = blockIdx.x * kTile, c0 = blockIdx.y * kTile;
  if (r0 >= m || c0 >= ncols) return;
  const long lda = D.lda;
  cplx* A = D.A;
  tile_gemm(m, ncols, jb, A + lda * j, lda, A + j + lda * n, lda, A + lda * n, lda, -1.0, 1.0, r0, c0, lds);
}

void launch_lu_multi(hipStream_t st, const LuDesc* d, int count, int nmax, int ncolmax, int nrhsmax) {
  if (count <= 0 || nmax <= 0) return;
  for (int j = 0; j < nmax; j += kNB) {
    hipLaunchKernelGGL(k_lu_panel, dim3(count), dim3(256), 0, st, d, j);
    // upper bounds over the batch: a matrix whose last panel is narrower than
    // kNB starts its trailing columns / rows before j + kNB
    const int rest = ncolmax - j - 1;
    if (ncolmax > 1)
      hipLaunchKernelGGL(k_lu_swap_trsm, dim3(cdiv_int(ncolmax, 64), count), dim3(256), 0, st, d, j);
    if (rest > 0) {
      const int mrest = nmax - j - 1;
      if (mrest > 0)
        hipLaunchKernelGGL(k_lu_update, dim3(cdiv_int(mrest, kTile), cdiv_int(rest, kTile), count), dim3(256), 0,
                           st, d, j);
    }
  }
  if (nrhsmax > 0) {
    const int nb0 = ((nmax - 1) / kNB) * kNB;
    for (int j = nb0; j >= 0; j -= kNB) {
      hipLaunchKernelGGL(k_lu_trsm_upper, dim3(cdiv_int(nrhsmax, 256), count), dim3(256), 0, st, d, j);
      if (j > 0)
        hipLaunchKernelGGL(k_lu_backupdate, dim3(cdiv_int(j, kTile), cdiv_int(nrhsmax, kTile), count), dim3(256),
                           0, st, d, j);
    }
  }
  HIPCHK(hipGetLastError());
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

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
constexpr int kNB = 16;  // LU panel width (register-resident panels)

// One 64 x (NT/4) tile of C = beta C + alpha A B computed by a workgroup of
// NT threads (16 x NT/16 threads, 4 x 4 accumulators each), staging 16-deep
// slices of both operands in LDS (64 x 16 and 16 x NT/4 complex).
template <int NT>
__device__ void tile_gemm_t(int m, int n, int k, const cplx* __restrict__ A, long lda, const cplx* __restrict__ B,
                            long ldb, cplx* __restrict__ C, long ldc, double alpha, double beta, int r0, int c0,
                            cplx* lds) {
  constexpr int TN = NT / 4;  // tile columns
  cplx* As = lds;             // [kKC][64]
  cplx* Bs = lds + kKC * 64;  // [kKC][TN]
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  cplx acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = mk(0, 0);
  for (int k0 = 0; k0 < k; k0 += kKC) {
#pragma unroll
    for (int q = 0; q < (kKC * 64) / NT; ++q) {
      const int e = tid + NT * q;
      const int row = e & 63, kk = e >> 6;
      const int gr = r0 + row, gk = k0 + kk;
      As[kk * 64 + row] = (gr < m && gk < k) ? A[gr + lda * gk] : mk(0, 0);
    }
#pragma unroll
    for (int q = 0; q < (kKC * TN) / NT; ++q) {
      const int e = tid + NT * q;
      const int kb = e & 15, col = e >> 4;
      const int gk2 = k0 + kb, gc = c0 + col;
      Bs[kb * TN + col] = (gk2 < k && gc < n) ? B[gk2 + ldb * gc] : mk(0, 0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kKC; ++kk) {
      cplx a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk * 64 + tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk * TN + ty + (NT / 16) * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) fma_acc(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int gc = c0 + ty + (NT / 16) * j;
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

__device__ inline void tile_gemm(int m, int n, int k, const cplx* A, long lda, const cplx* B, long ldb, cplx* C,
                                 long ldc, double alpha, double beta, int r0, int c0, cplx* lds) {
  tile_gemm_t<256>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, r0, c0, lds);
}

// Whole GEMM by one workgroup of NT threads (loops over its tiles).
template <int NT>
__device__ void wg_gemm_t(int m, int n, int k, const cplx* A, long lda, const cplx* B, long ldb, cplx* C, long ldc,
                          double alpha, double beta, cplx* lds) {
  if (m <= 0 || n <= 0) return;
  constexpr int TN = NT / 4;
  for (int c0 = 0; c0 < n; c0 += TN)
    for (int r0 = 0; r0 < m; r0 += 64) tile_gemm_t<NT>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, r0, c0, lds);
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
  // sval / sidx hold at least blockDim.x / 64 + 1 entries
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nt = blockDim.x, nw = nt >> 6;
  double best = -1.0;
  int bi = lo;
  for (int i = lo + tid; i < hi; i += nt) {
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
    for (int w = 1; w < nw; ++w)
      if (sval[w] > b || (sval[w] == b && sidx[w] < ix)) { b = sval[w]; ix = sidx[w]; }
    sval[16] = b;
    sidx[16] = ix;
  }
  __syncthreads();
  piv = sidx[16];
  pval = sval[16];
  __syncthreads();
}

// Factor the panel A[j:n, j:j+jb] with partial pivoting; row interchanges are
// applied inside the panel only (the caller applies them to the other columns).
__device__ void wg_lu_panel(const LuDesc& D, int j, int jb, double* sval, int* sidx) {
  __shared__ cplx urow[kNB];
  __shared__ int pivs[kNB];
  __shared__ int sing;
  if (threadIdx.x == 0) sing = -1;
  __syncthreads();
  const int n = D.n;
  const long lda = D.lda;
  cplx* A = D.A;
  const int tid = threadIdx.x;
  for (int jj = j; jj < j + jb; ++jj) {
    int p;
    double pv;
    wg_argmax_abs(A + lda * jj, jj, n, p, pv, sval, sidx);
    if (tid == 0) {
      pivs[jj - j] = p;
      if (pv == 0.0 && sing < 0) sing = jj;
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
    for (int i = jj + 1 + tid; i < n; i += (int)blockDim.x) {
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
  if (tid < jb) D.ipiv[j + tid] = pivs[tid];
  if (tid == 0 && sing >= 0 && *D.info == 0) *D.info = sing + 1;
  __syncthreads();
}


// Panel factorisation with the panel held in registers: thread t owns panel
// rows j + t + NT q (q < R), all JB columns.  Per column: arg-max of the
// owned rows, a workgroup reduction, the two interchanged rows swapped
// through LDS, then scaling and the rank-1 update in registers.  No global
// memory traffic inside the column loop.  The column loop is unrolled by a
// compile-time recursion so that every register index is a constant.
// Requires n - j <= NT R and jb <= JB.
struct RegPanelCtx {
  const LuDesc* D;
  int j, jb, n;
  double* sval;
  int* sidx;
  cplx* rowP;
  cplx* rowJ;
  int* pivs;  // LDS: the panel's pivot rows
  int* sing;  // LDS: first zero pivot (-1: none)
};

template <int CC, int NT, int R, int JB>
struct RegPanelStep {
  // Two barriers per column: the reduction slots and the two exchanged rows
  // alternate between two LDS buffers, so the next column may overwrite one
  // buffer while a slow wavefront still reads the other.
  static __device__ __forceinline__ void run(const RegPanelCtx& X, cplx (&a)[R][JB]) {
    if (CC < X.jb) {
      const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
      constexpr int NW = NT / 64;
      constexpr int B = CC & 1;
      double* sval = X.sval + 17 * B;
      int* sidx = X.sidx + 17 * B;
      cplx* rowP = X.rowP + JB * B;
      cplx* rowJ = X.rowJ + JB * B;
      const int j = X.j, n = X.n, jj = j + CC;
      double best = -1.0;
      int bi = jj;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = j + tid + NT * q;
        const double v = abs2(a[q][CC]);
        if (i >= jj && i < n && v > best) { best = v; bi = i; }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) { sval[wave] = best; sidx[wave] = bi; }
      __syncthreads();
      // every thread combines the per-wavefront candidates itself
      double pv = sval[0];
      int p = sidx[0];
#pragma unroll
      for (int w = 1; w < NW; ++w)
        if (sval[w] > pv || (sval[w] == pv && sidx[w] < p)) { pv = sval[w]; p = sidx[w]; }
      if (tid == 0) {
        X.pivs[CC] = p;  // written to global memory after the panel
        if (pv == 0.0 && *X.sing < 0) *X.sing = jj;
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = j + tid + NT * q;
        if (i == p) {
#pragma unroll
          for (int c = 0; c < JB; ++c) rowP[c] = a[q][c];
        }
        if (i == jj) {
#pragma unroll
          for (int c = 0; c < JB; ++c) rowJ[c] = a[q][c];
        }
      }
      __syncthreads();
      const cplx inv = (pv == 0.0) ? mk(0, 0) : cdiv(mk(1, 0), rowP[CC]);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = j + tid + NT * q;
        if (i == jj) {
#pragma unroll
          for (int c = 0; c < JB; ++c) a[q][c] = rowP[c];
        } else {
          if (i == p) {
#pragma unroll
            for (int c = 0; c < JB; ++c) a[q][c] = rowJ[c];
          }
          if (i > jj && i < n) {
            const cplx l = a[q][CC] * inv;
            a[q][CC] = l;
#pragma unroll
            for (int c = CC + 1; c < JB; ++c) {
              const cplx u = rowP[c];
              a[q][c].re -= l.re * u.re - l.im * u.im;
              a[q][c].im -= l.re * u.im + l.im * u.re;
            }
          }
        }
      }
    }
    RegPanelStep<CC + 1, NT, R, JB>::run(X, a);
  }
};

template <int NT, int R, int JB>
struct RegPanelStep<JB, NT, R, JB> {
  static __device__ __forceinline__ void run(const RegPanelCtx&, cplx (&)[R][JB]) {}
};

template <int NT, int R, int JB>
__device__ void reg_lu_panel(const LuDesc& D, int j, int jb, double* sval, int* sidx, cplx* rowP, cplx* rowJ) {
  const int n = D.n;
  const long lda = D.lda;
  cplx* A = D.A;
  const int tid = threadIdx.x;
  cplx a[R][JB];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = j + tid + NT * q;
#pragma unroll
    for (int c = 0; c < JB; ++c) a[q][c] = (i < n && c < jb) ? A[i + lda * (j + c)] : mk(0, 0);
  }
  __shared__ int pivs[JB];
  __shared__ int sing;
  if (tid == 0) sing = -1;
  __syncthreads();
  const RegPanelCtx X{&D, j, jb, n, sval, sidx, rowP, rowJ, pivs, &sing};
  RegPanelStep<0, NT, R, JB>::run(X, a);
  __syncthreads();
  if (tid < jb) D.ipiv[j + tid] = pivs[tid];
  if (tid == 0 && sing >= 0 && *D.info == 0) *D.info = sing + 1;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = j + tid + NT * q;
    if (i < n) {
#pragma unroll
      for (int c = 0; c < JB; ++c)
        if (c < jb) A[i + lda * (j + c)] = a[q][c];
    }
  }
}


// Panel of at most MAXR rows factored by wavefront 0 alone, out of LDS
// (P: JB columns x MAXR rows).  Within one wavefront no workgroup barrier is
// needed: the arg-max is a shuffle reduction and LDS accesses of a wavefront
// complete in order (made explicit with wavefront-scope fences).
template <int MAXR, int JB>
__device__ void wave_lu_panel(const LuDesc& D, int j, int jb, cplx* P) {
  __shared__ int pivs[JB];
  __shared__ int sing;
  const int n = D.n;
  const long lda = D.lda;
  cplx* A = D.A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rows = n - j;
  for (int q = tid; q < JB * MAXR; q += blockDim.x) {
    const int r = q % MAXR, c = q / MAXR;
    P[q] = (r < rows && c < jb) ? A[j + r + lda * (j + c)] : mk(0, 0);
  }
  if (tid == 0) sing = -1;
  __syncthreads();
  if (wave == 0) {
    for (int cc = 0; cc < jb; ++cc) {
      double best = -1.0;
      int bi = cc;
      for (int r = cc + lane; r < rows; r += 64) {
        const double v = abs2(P[cc * MAXR + r]);
        if (v > best) { best = v; bi = r; }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      const int p = bi;
      // pivots and the singularity flag stay in LDS until the panel is done:
      // a global store here would make every fence wait for its completion
      if (lane == 0) {
        pivs[cc] = j + p;
        if (best == 0.0 && sing < 0) sing = j + cc;
      }
      if (lane < jb && p != cc) {
        const cplx t = P[lane * MAXR + cc];
        P[lane * MAXR + cc] = P[lane * MAXR + p];
        P[lane * MAXR + p] = t;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const cplx inv = (best == 0.0) ? mk(0, 0) : cdiv(mk(1, 0), P[cc * MAXR + cc]);
      // pivot row to the right of cc in registers (zero elsewhere), then each
      // row is updated over all JB columns without branches: its loads are
      // independent and issue back to back
      cplx u[JB];
#pragma unroll
      for (int c = 0; c < JB; ++c) {
        const cplx t = P[c * MAXR + cc];
        u[c] = (c > cc) ? t : mk(0, 0);
      }
      for (int r = cc + 1 + lane; r < rows; r += 64) {
        cplx x[JB];
#pragma unroll
        for (int c = 0; c < JB; ++c) x[c] = P[c * MAXR + r];
        const cplx l = P[cc * MAXR + r] * inv;
#pragma unroll
        for (int c = 0; c < JB; ++c) {
          x[c].re -= l.re * u[c].re - l.im * u[c].im;
          x[c].im -= l.re * u[c].im + l.im * u[c].re;
        }
#pragma unroll
        for (int c = 0; c < JB; ++c) P[c * MAXR + r] = x[c];
        P[cc * MAXR + r] = l;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int q = tid; q < JB * MAXR; q += blockDim.x) {
    const int r = q % MAXR, c = q / MAXR;
    if (r < rows && c < jb) A[j + r + lda * (j + c)] = P[q];
  }
  if (tid < jb) D.ipiv[j + tid] = pivs[tid];
  if (tid == 0 && sing >= 0 && *D.info == 0) *D.info = sing + 1;
}



// Net row permutation of panel [j, j+jb): after the panel's interchanges
// (ipiv[j..j+jb-1], applied in order) row prow[t] holds the former row
// porig[t], for t < *pm.  Touched rows are j..j+jb-1 and the pivot rows; at
// most 2 kNB entries.  Computed by one thread into LDS.
__device__ void panel_perm(const LuDesc& D, int j, int jb, int* prow, int* porig, int* pm) {
  int m = 0;
  for (int t = 0; t < jb; ++t) {
    prow[m] = j + t;
    porig[m] = j + t;
    ++m;
  }
  for (int jj = j; jj < j + jb; ++jj) {
    const int p = D.ipiv[jj];
    if (p == jj) continue;
    int ip = -1;
    for (int t = 0; t < m; ++t)
      if (prow[t] == p) ip = t;
    if (ip < 0) {
      prow[m] = p;
      porig[m] = p;
      ip = m++;
    }
    const int ij = jj - j;
    const int tmp = porig[ij];
    porig[ij] = porig[ip];
    porig[ip] = tmp;
  }
  *pm = m;
}

// One column c outside the panel: gather the touched rows into registers
// (independent loads), then - for columns right of the panel - solve with the
// unit lower triangular L11 (in LDS, JB x JB column-major) and write back.
template <int JB>
__device__ inline void perm_trsm_column(const LuDesc& D, int j, int jb, int c, bool solve, const int* prow,
                                        const int* porig, int m, const cplx* L11) {
  const long lda = D.lda;
  cplx* col = D.A + lda * c;
  cplx v[2 * JB];
#pragma unroll
  for (int t = 0; t < 2 * JB; ++t) v[t] = (t < m) ? col[porig[t]] : mk(0, 0);
  if (solve) {
    // rows j..j+jb-1 are the first jb touched rows
#pragma unroll
    for (int r = 1; r < JB; ++r) {
      if (r < jb) {
        cplx s = v[r];
#pragma unroll
        for (int l = 0; l < r; ++l) {
          const cplx L = L11[r + JB * l];
          s.re -= L.re * v[l].re - L.im * v[l].im;
          s.im -= L.re * v[l].im + L.im * v[l].re;
        }
        v[r] = s;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 2 * JB; ++t)
    if (t < m) col[prow[t]] = v[t];
}

// Backward substitution on one appended column for block row [j, j+jb) with
// the upper triangular block U (in LDS, JB x JB column-major).
template <int JB>
__device__ inline void backsub_column(const LuDesc& D, int j, int jb, int c, const cplx* U) {
  const long lda = D.lda;
  cplx* col = D.A + lda * c + j;
  cplx x[JB];
#pragma unroll
  for (int r = 0; r < JB; ++r) x[r] = (r < jb) ? col[r] : mk(0, 0);
#pragma unroll
  for (int r = JB - 1; r >= 0; --r) {
    if (r < jb) {
      cplx s = x[r];
#pragma unroll
      for (int l = r + 1; l < JB; ++l) {
        if (l < jb) {
          const cplx u = U[r + JB * l];
          s.re -= u.re * x[l].re - u.im * x[l].im;
          s.im -= u.re * x[l].im + u.im * x[l].re;
        }
      }
      x[r] = cdiv(s, U[r + JB * r]);
    }
  }
#pragma unroll
  for (int r = 0; r < JB; ++r)
    if (r < jb) col[r] = x[r];
}

__device__ inline void stage_block(const LuDesc& D, int j, int jb, cplx* dst) {
  for (int q = threadIdx.x; q < kNB * kNB; q += blockDim.x) {
    const int r = q % kNB, c = q / kNB;
    dst[q] = (r < jb && c < jb) ? D.A[j + r + (long)D.lda * (j + c)] : mk(r == c ? 1.0 : 0.0, 0.0);
  }
}

// Right-looking blocked LU with partial pivoting of A[0:n, 0:n] with row
// interchanges applied to all ncol columns, then backward substitution on
// the appended columns: on exit A[0:n, n:ncol] = D^{-1} (original appended
// columns).  One workgroup per matrix.
constexpr int kLuThreads = 512;  // 8 wavefronts: 2 per SIMD fit the 254-VGPR kernel

__global__ __launch_bounds__(kLuThreads) void k_lu_fused(const LuDesc* __restrict__ descs) {
  __shared__ cplx lds[kKC * 64 + kKC * kLuThreads / 4];
  __shared__ double sval[17];
  __shared__ int sidx[17];
  __shared__ cplx Ppanel[kNB * 256];
  __shared__ cplx Blk[kNB * kNB];
  __shared__ int prow[2 * kNB], porig[2 * kNB], pm;
  const LuDesc D = descs[blockIdx.x];
  const int n = D.n, nc = D.ncol;
  const long lda = D.lda;
  cplx* A = D.A;
  const int tid = threadIdx.x;
  for (int j = 0; j < n; j += kNB) {
    const int jb = min(kNB, n - j);
    if (n - j <= 256) wave_lu_panel<256, kNB>(D, j, jb, Ppanel);
    else wg_lu_panel(D, j, jb, sval, sidx);
    __syncthreads();
    if (tid == 0) panel_perm(D, j, jb, prow, porig, &pm);
    stage_block(D, j, jb, Blk);
    __syncthreads();
    for (int e = tid; e < nc - jb; e += kLuThreads) {
      const int c = e < j ? e : e + jb;
      perm_trsm_column<kNB>(D, j, jb, c, c >= j + jb, prow, porig, pm, Blk);
    }
    __syncthreads();
    wg_gemm_t<kLuThreads>(n - j - jb, nc - j - jb, jb, A + (j + jb) + lda * j, lda, A + j + lda * (j + jb), lda,
            A + (j + jb) + lda * (j + jb), lda, -1.0, 1.0, lds);
    __syncthreads();
  }
  if (nc == n) return;
  // backward substitution with U on the appended columns, blocked from the bottom
  const int nb0 = ((n - 1) / kNB) * kNB;
  for (int j = nb0; j >= 0; j -= kNB) {
    const int jb = min(kNB, n - j);
    stage_block(D, j, jb, Blk);
    __syncthreads();
    for (int c = n + tid; c < nc; c += kLuThreads) backsub_column<kNB>(D, j, jb, c, Blk);
    __syncthreads();
    wg_gemm_t<kLuThreads>(j, nc - n, jb, A + lda * j, lda, A + j + lda * n, lda, A + lda * n, lda, -1.0, 1.0, lds);
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

constexpr int kNBM = kNB;  // panel width of the multi-workgroup path

// One workgroup per matrix; the block size picks the register layout: 1024
// threads x 1 row (<= 1024 rows) or 512 threads x 3 rows (<= 1536 rows),
// else the panel is factored in global memory.
template <int NT>
__global__ __launch_bounds__(NT) void k_lu_panel(const LuDesc* __restrict__ descs, int j) {
  __shared__ double sval[34];
  __shared__ int sidx[34];
  __shared__ cplx rowP[2 * kNBM], rowJ[2 * kNBM];
  const LuDesc D = descs[blockIdx.x];
  if (j >= D.n) return;
  const int jb = min(kNBM, D.n - j);
  const int rows = D.n - j;
  if (NT == 1024 && rows <= 1024) reg_lu_panel<NT, 1, kNBM>(D, j, jb, sval, sidx, rowP, rowJ);
  else if (NT == 512 && rows <= 1536) reg_lu_panel<NT, 3, kNBM>(D, j, jb, sval, sidx, rowP, rowJ);
  else wg_lu_panel(D, j, jb, sval, sidx);
}

// Columns outside panel [j, j+jb), one per thread: the panel's net row
// permutation (independent gathers), and for columns right of the panel
// U12 = L11^{-1} A12 in registers.
__global__ __launch_bounds__(256) void k_lu_swap_trsm(const LuDesc* __restrict__ descs, int j) {
  __shared__ cplx Blk[kNB * kNB];
  __shared__ int prow[2 * kNB], porig[2 * kNB], pm;
  const LuDesc D = descs[blockIdx.y];
  const int n = D.n, nc = D.ncol;
  if (j >= n) return;
  const int jb = min(kNBM, n - j);
  if (blockIdx.x * 256 >= nc - jb) return;
  if (threadIdx.x == 0) panel_perm(D, j, jb, prow, porig, &pm);
  stage_block(D, j, jb, Blk);
  __syncthreads();
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nc - jb) return;
  const int c = e < j ? e : e + jb;
  perm_trsm_column<kNB>(D, j, jb, c, c >= j + jb, prow, porig, pm, Blk);
}

// A22 -= L21 U12, one 64 x 64 tile per workgroup.
__global__ __launch_bounds__(256) void k_lu_update(const LuDesc* __restrict__ descs, int j) {
  __shared__ cplx lds[2 * kKC * kTile];
  const LuDesc D = descs[blockIdx.z];
  const int n = D.n, nc = D.ncol;
  if (j >= n) return;
  const int jb = min(kNBM, n - j);
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
  __shared__ cplx Blk[kNB * kNB];
  const LuDesc D = descs[blockIdx.y];
  const int n = D.n, nc = D.ncol;
  if (j >= n || nc == n) return;
  const int jb = min(kNBM, n - j);
  stage_block(D, j, jb, Blk);
  __syncthreads();
  const int c = n + blockIdx.x * 256 + threadIdx.x;
  if (c >= nc) return;
  backsub_column<kNB>(D, j, jb, c, Blk);
}

__global__ __launch_bounds__(256) void k_lu_backupdate(const LuDesc* __restrict__ descs, int j) {
  __shared__ cplx lds[2 * kKC * kTile];
  const LuDesc D = descs[blockIdx.z];
  const int n = D.n, nc = D.ncol;
  if (j >= n || nc == n) return;
  const int jb = min(kNBM, n - j);
  const int m = j, ncols = nc - n;
  const int r0 = blockIdx.x * kTile, c0 = blockIdx.y * kTile;
  if (r0 >= m || c0 >= ncols) return;
  const long lda = D.lda;
  cplx* A = D.A;
  tile_gemm(m, ncols, jb, A + lda * j, lda, A + j + lda * n, lda, A + lda * n, lda, -1.0, 1.0, r0, c0, lds);
}

void launch_lu_multi(hipStream_t st, const LuDesc* d, int count, int nmax, int ncolmax, int nrhsmax) {
  if (count <= 0 || nmax <= 0) return;
  for (int j = 0; j < nmax; j += kNBM) {
    const int rows = nmax - j;
    if (rows <= 1024) hipLaunchKernelGGL(k_lu_panel<1024>, dim3(count), dim3(1024), 0, st, d, j);
    else if (rows <= 1536) hipLaunchKernelGGL(k_lu_panel<512>, dim3(count), dim3(512), 0, st, d, j);
    else hipLaunchKernelGGL(k_lu_panel<256>, dim3(count), dim3(256), 0, st, d, j);
    // upper bounds over the batch: a matrix whose last panel is narrower than
    // the panel width starts its trailing columns / rows before j + kNB
    const int rest = ncolmax - j - 1;
    if (ncolmax > 1)
      hipLaunchKernelGGL(k_lu_swap_trsm, dim3(cdiv_int(ncolmax, 256), count), dim3(256), 0, st, d, j);
    if (rest > 0) {
      const int mrest = nmax - j - 1;
      if (mrest > 0)
        hipLaunchKernelGGL(k_lu_update, dim3(cdiv_int(mrest, kTile), cdiv_int(rest, kTile), count), dim3(256), 0,
                           st, d, j);
    }
  }
  if (nrhsmax > 0) {
    const int nb0 = ((nmax - 1) / kNBM) * kNBM;
    for (int j = nb0; j >= 0; j -= kNBM) {
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
  hipLaunchKernelGGL(k_lu_fused, dim3(count), dim3(kLuThreads), 0, st, d);
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

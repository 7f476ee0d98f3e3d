// Descriptors and launchers of the HIP kernels, shared by the kernels and
// the host driver.
#pragma once

#include "common.hpp"

namespace symhss {

struct IdDesc {
  cplx* A;
  int m, n, ld;
  int target;   // < 0: tolerance mode; >= 0: factor up to this rank (resume)
  int* perm;    // n entries
  int* rank;    // in: steps already done (resume), out: rank
  double* r00;  // |R_00|
};

// Dense interpolation matrix of one half: out[row0 + r, col0 + perm[c]] =
// (c < k ? delta_rc : T[r, c - k]) for the column ID (R = [I T] P^T), or the
// transposed placement out[col0 + perm[c], row0 + r] for a row ID (L = R^T;
// plain transpose, no conjugate).  The output must be zeroed beforehand.
struct InterpDesc {
  const cplx* A;  // T lives in A[0:k, k:n]
  int ld, k, n;
  const int* perm;
  cplx* out;
  int ldo, row0, col0, transpose;
};

struct LuDesc {
  cplx* A;
  int n;     // order of the factored block
  int ncol;  // total columns (n + appended right-hand sides)
  int lda;
  int* ipiv;
  int* info;
};

struct GemmDesc {
  const cplx* A;
  const cplx* B;
  cplx* C;
  int m, n, k;
  int lda, ldb, ldc;
  double alpha, beta;  // real scalars: C = beta C + alpha A B
};

struct CopyDesc {
  // dst[dmap[i] + ldd * c] = src[smap[i] + lds * c], i < rows, c < cols;
  // a null map means the identity.
  const cplx* src;
  cplx* dst;
  const int* smap;
  const int* dmap;
  int rows, cols, lds, ldd;
};

struct Scatter2Desc {
  // dst[rmap[i] + ldd * cmap[j]] = src[i + lds * j]
  const cplx* src;
  cplx* dst;
  const int* rmap;
  const int* cmap;
  int m, n, lds, ldd;
};

// Solve with a factored block for a few right-hand sides held apart from the
// factor: B := D^{-1} B using the pivots and L, U of k_lu_fused.
struct SolveDesc {
  const cplx* LU;
  const int* ipiv;
  cplx* B;
  int n, lda, ldb, nrhs;
};

// kernel-block generation (kblock.hip)
// media: device array indexed by KJob::med
void launch_kblock(hipStream_t st, const PointsDev& P, const MediumDev* media, const KJob* jobs,
                   const KTile* tiles, int ntiles, const int* rpt, const int* rmap1, const int* rmap2,
                   const int* cpt, const int* cmap1, const int* cmap2);
void launch_geometry(hipStream_t st, int n, const double* x, const double* dx, const double* ddx, double* px,
                     double* py, double* nx, double* ny, double* w, double* kappa);
void launch_rhs_plane(hipStream_t st, int n, const PointsDev& P, const MediumDev& md, double angle, cplx* b);
void launch_bessel(hipStream_t st, int n, const double* z, double* out);
void launch_matvec_direct(hipStream_t st, const PointsDev& P, const MediumDev& md, const cplx* x, cplx* y);

// interpolative decomposition (cpqr.hip)
size_t cpqr_lds_bytes(int mmax, int nmax);
struct CpqrVariant {
  int threads = 256;   // 256 or 1024 per workgroup
  int persistent = 0;  // 1: work-queue grid (needs a device counter)
};
CpqrVariant cpqr_default_variant(int count);
// queue: one device int, used (and zeroed first) by persistent variants
void launch_cpqr(hipStream_t st, const IdDesc* descs, int count, int mmax, int nmax, double tol, int want_T,
                 const CpqrVariant& var, int* queue);
void launch_build_interp(hipStream_t st, const InterpDesc* descs, int count, int nmax);
void launch_equalise_ranks(hipStream_t st, int npairs, const int* ia, const int* ib, IdDesc* descs);

// one-thread-per-element int zeroing (graph-safe, no memset node)
__global__ void k_zero_i32(int* p, int n);

// batched dense algebra (dense.hip)
void launch_lu_fused(hipStream_t st, const LuDesc* d, int count);
// host-looped multi-workgroup variant; nmax / ncolmax / nrhsmax bound n, ncol, ncol - n
void launch_lu_multi(hipStream_t st, const LuDesc* d, int count, int nmax, int ncolmax, int nrhsmax);
void launch_gemm_batched(hipStream_t st, const GemmDesc* d, int count, int mmax, int nmax);
void launch_lu_solve(hipStream_t st, const SolveDesc* d, int count);
void launch_copy_batched(hipStream_t st, const CopyDesc* d, int count, long maxelems);
void launch_scatter2_batched(hipStream_t st, const Scatter2Desc* d, int count, long maxelems);
void launch_zero(hipStream_t st, cplx* p, long count);
void launch_set_identity(hipStream_t st, const LuDesc* d, int count, int nmax);

}  // namespace symhss

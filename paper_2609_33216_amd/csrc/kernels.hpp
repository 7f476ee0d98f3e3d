// Descriptors and launchers of the HIP kernels, shared by the kernels and
// the host driver.
#pragma once

#include <algorithm>

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
  const cplx* A;  // column c >= k of T lives in A[0:k, perm[c]]
  int ld, k, n;
  const int* perm;
  cplx* out;
  int ldo, row0, col0, transpose;
};

#include "dense_types.inc"

// kernel-block generation (kblock.hip)
// media: device array indexed by KJob::med
void launch_kblock(hipStream_t st, int eq, const PointsDev& P, const MediumDev* media, const KJob* jobs,
                   const KTile* tiles, int ntiles, const int* rpt, const int* rmap1, const int* rmap2,
                   const int* cpt, const int* cmap1, const int* cmap2);
void launch_geometry(hipStream_t st, int n, const double* x, const double* dx, const double* ddx, double* px,
                     double* py, double* nx, double* ny, double* w, double* kappa);
void launch_rhs_plane(hipStream_t st, int n, const PointsDev& P, const MediumDev& md, double angle, cplx* b);
// u_in and q_in = du_in/dnu of the plane wave at the n nodes of P
void launch_plane_incident(hipStream_t st, int n, const PointsDev& P, const MediumDev& md, double angle, cplx* uin,
                           cplx* qin);
// right-hand sides of md's system from nrhs columns of traces (leading dimension ldi) into b (ldb)
void launch_rhs_incident(hipStream_t st, int n, const PointsDev& P, const MediumDev& md, const cplx* uin,
                         const cplx* qin, int ldi, cplx* b, int ldb, int nrhs);
// solution columns [q; u] of one boundary (ldx) -> traces q and u (ldo)
void launch_split_traces(hipStream_t st, int n, const cplx* x, int ldx, cplx* q, cplx* u, int ldo, int nrhs);
void launch_bessel(hipStream_t st, int n, const double* z, double* out);
void launch_matvec_direct(hipStream_t st, const PointsDev& P, const MediumDev& md, const cplx* x, cplx* y);

// interpolative decomposition (cpqr.hip)
size_t cpqr_lds_bytes(int mmax, int nmax);
struct CpqrVariant {
  int threads = 256;   // 256 or 1024 per workgroup
  int persistent = 0;  // 1: work-queue grid (needs a device counter)
  int qr = 0;          // 1: blocked QR, then pivoted QR of the triangle in registers (idqr.hip)
};
CpqrVariant cpqr_default_variant(int count, int mmax, int nmax);
// queue: one device int, used (and zeroed first) by persistent variants;
// resume: a pass that continues the IDs a previous launch of the same
// variant stopped (targets set, rank = steps done)
void launch_cpqr(hipStream_t st, const IdDesc* descs, int count, int mmax, int nmax, double tol, int want_T,
                 const CpqrVariant& var, int* queue, bool resume);
// the two-stage ID of idqr.hip: matrices of at most 128 columns and 512 rows
bool id_qr_eligible(int mmax, int nmax);
void launch_id_qr(hipStream_t st, const IdDesc* descs, int count, int mmax, int nmax, double tol, int want_T,
                  bool resume);
void launch_build_interp(hipStream_t st, const InterpDesc* descs, int count, int nmax);
void launch_equalise_ranks(hipStream_t st, int npairs, const int* ia, const int* ib, IdDesc* descs);

// one-thread-per-element int zeroing (graph-safe, no memset node)
__global__ void k_zero_i32(int* p, int n);

// batched dense algebra (dense.hip)
#include "dense_api.inc"

// mixed precision (mixed.hip): FP64 -> FP32 block copies and FP64 refinement vectors
struct ConvDesc {
  // dst[i + ldd c] = (FP32) src[i + lds c], i < rows, c < cols
  const cplx* src;
  cplxf* dst;
  int rows, cols, lds, ldd;
};
void launch_convert_batched(hipStream_t st, const ConvDesc* d, int count, long maxelems);
// FP32 blocks placed in an FP64 matrix: dst[rmap[i] + ldd cmap[j]] = src[i + lds j]
struct Scatter2WideDesc {
  const cplxf* src;
  cplx* dst;
  const int* rmap;
  const int* cmap;
  int m, n, lds, ldd;
};
void launch_scatter2_widen(hipStream_t st, const Scatter2WideDesc* d, int count, long maxelems);
// descriptor upload from pinned staging memory by a copy kernel (upload.hip)
void launch_upload(hipStream_t st, void* dst, const void* src_pinned, size_t bytes);
// na arrays of n doubles, back to back in pinned staging: array a to dst + a ld
void launch_upload_split(hipStream_t st, double* dst, size_t ld, const double* src_pinned, size_t n, int na);
void launch_round_vec(hipStream_t st, const cplx* x, cplxf* y, long n);
void launch_add_vec(hipStream_t st, cplx* x, const cplxf* d, long n);
void launch_widen_vec(hipStream_t st, const cplxf* x, cplx* y, long n);
void launch_sub_vec(hipStream_t st, const cplx* b, const cplx* y, cplx* r, long n);
// squared 2-norms of ncols columns; work holds kNormParts doubles per column
constexpr int kNormParts = 64;
void launch_col_norm2(hipStream_t st, const cplx* v, long n, long ld, int ncols, double* out, double* work);

// the same in complex FP32 (dense32.hip)
namespace f32 {
using cplx = cplxf;
__host__ __device__ inline cplx mk(double r, double i) { return cplx{(float)r, (float)i}; }
#include "dense_types.inc"
#include "dense_api.inc"
}  // namespace f32

}  // namespace symhss

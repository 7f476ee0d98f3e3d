// Interpolative decomposition of proxy matrices by column-pivoted
// Householder QR (paper Section 4.1: the ID of each half of M_R, and for the
// two-sided baseline of each half of M_L^T).
//
// For M (m x n, column-major, in place): M P = Q R.  Pivot j is the remaining
// column of largest trailing norm (lowest position on ties); trailing norms are
// recomputed exactly while each column is updated, so no downdating error
// accumulates.  The rank k is the first j with |R_jj| <= tol |R_00|
// (tolerance mode) or a fixed target (resume mode, used to equalise row and
// column ranks in the two-sided baseline).  Afterwards (want_T) T = R11^{-1}
// R12 overwrites R12, so that M[:, P[k:]] ~= M[:, P[:k]] T; a pass that may
// be resumed leaves R12 in place.  Columns are not moved: column t of R (or
// T) is stored in the memory of original column perm[t].
//
// One workgroup per matrix.  The Householder vector of the current step is
// staged in LDS; every wavefront then takes groups of trailing columns,
// forms v^H a_c with wavefront reductions, applies the reflector and
// recomputes the columns' trailing norms in the same pass.
#include <algorithm>

#include "kernels.hpp"

namespace symhss {


__global__ void k_zero_i32(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__device__ inline double wave_sum(double v) { return wave_sum_dpp(v); }

// Apply the step's reflector H = I - tau v v^H to the nc <= CB columns
// pc[0..nc) (physical indices) over rows j..m-1 and recompute their norms
// below row j.  The column segments (R*64 rows per column) are loaded into
// registers together, so one wavefront keeps CB*R loads in flight.
template <int R, int CB>
__device__ inline void reflect_columns(const IdDesc& D, int j, const int* pc, int nc, const cplx* __restrict__ vj,
                                       double tau, double* vn, int lane) {
  const long ld = D.ld;
  const int rows = D.m - j;
  cplx a[CB][R];
  cplx w[CB];
  int c[CB];
#pragma unroll
  for (int b = 0; b < CB; ++b) c[b] = b < nc ? pc[b] : -1;
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    const cplx* col = D.A + ld * (c[b] >= 0 ? c[b] : 0) + j;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = lane + 64 * q;
      a[b][q] = (c[b] >= 0 && i < rows) ? ldg(col + i) : mk(0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    w[b] = mk(0, 0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = lane + 64 * q;
      if (i < rows) fma_conj_acc(w[b], vj[i], a[b][q]);
    }
  }
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    w[b].re = wave_sum_dpp(w[b].re);
    w[b].im = wave_sum_dpp(w[b].im);
  }
  double s[CB];
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    const cplx tw = tau * w[b];
    cplx* col = D.A + ld * (c[b] >= 0 ? c[b] : 0) + j;
    s[b] = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = lane + 64 * q;
      if (c[b] >= 0 && i < rows) {
        const cplx vi = vj[i];
        a[b][q].re -= vi.re * tw.re - vi.im * tw.im;
        a[b][q].im -= vi.re * tw.im + vi.im * tw.re;
        stg(col + i, a[b][q]);
        if (i > 0) s[b] += abs2(a[b][q]);
      }
    }
  }
#pragma unroll
  for (int b = 0; b < CB; ++b) s[b] = wave_sum_dpp(s[b]);
  if (lane == 0) {
#pragma unroll
    for (int b = 0; b < CB; ++b)
      if (c[b] >= 0) vn[c[b]] = s[b];
  }
}

// One column (physical index c), any number of rows (streamed from global
// memory).
__device__ inline void reflect_column_long(const IdDesc& D, int j, int c, const cplx* __restrict__ vj, double tau,
                                           double* vn, int lane) {
  const int rows = D.m - j;
  cplx* col = D.A + (long)D.ld * c + j;
  cplx w = mk(0, 0);
  for (int i = lane; i < rows; i += 64) fma_conj_acc(w, vj[i], ldg(col + i));
  w.re = wave_sum(w.re);
  w.im = wave_sum(w.im);
  const cplx tw = tau * w;
  double s = 0.0;
  for (int i = lane; i < rows; i += 64) {
    cplx a = ldg(col + i);
    const cplx vi = vj[i];
    a.re -= vi.re * tw.re - vi.im * tw.im;
    a.im -= vi.re * tw.im + vi.im * tw.re;
    stg(col + i, a);
    if (i > 0) s += abs2(a);
  }
  s = wave_sum(s);
  if (lane == 0) vn[c] = s;
}

// The ID of one matrix by one workgroup of NT threads.
//
// Column interchanges are logical: columns stay where they are in memory and
// pos[t] (in LDS, copied to D.perm at the end) names the column at position
// t, so column t of the factored matrix - R, or T after want_T - lives at
// A[:, perm[t]].  A resumed pass starts from the stored perm.  The pivot
// choice is made by every thread from the per-wavefront candidates, which
// leaves two workgroup barriers per step.
template <int NT, int R, int CB>
__device__ void cpqr_one(const IdDesc& D, double tol, int want_T, double* lds) {
  const int m = D.m, n = D.n;
  const long ld = D.ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int nwaves = NT / 64;
  // LDS: vn[n] doubles (by physical column), v[m] complex, reduction
  // scratch, pos[n] ints
  double* vn = lds;
  cplx* v = reinterpret_cast<cplx*>(lds + n);
  double* red = lds + n + 2 * m;                     // nwaves doubles
  int* redi = reinterpret_cast<int*>(red + nwaves);  // nwaves ints
  int* pos = redi + nwaves;                          // n ints
  __shared__ double s_tau;

  const int kmax = m < n ? m : n;
  const int j0 = (D.target >= 0) ? ldg(D.rank) : 0;
  for (int c = tid; c < n; c += NT) pos[c] = (j0 == 0) ? c : ldg(D.perm + c);
  __syncthreads();
  // trailing norms over rows j0..m-1 of the columns not yet pivoted
  for (int t = j0 + wave; t < n; t += nwaves) {
    const int c = pos[t];
    const cplx* col = D.A + ld * c;
    double s = 0.0;
    for (int i = j0 + lane; i < m; i += 64) s += abs2(ldg(col + i));
    s = wave_sum(s);
    if (lane == 0) vn[c] = s;
  }
  __syncthreads();
  double r00 = (j0 > 0) ? ldg(D.r00) : 0.0;
  int j = j0;
  for (; j < kmax; ++j) {
    // pivot: the position t >= j of largest trailing norm.  Each thread's
    // best position exactly (lowest t on ties), then 32-bit arg-max keys over
    // the wavefront (the lane in the key: norms equal to about 2^-13 relative
    // go to the lowest lane) and over the wavefronts (lowest wavefront)
    double best = -1.0;
    int bt = n;
    for (int t = j + tid; t < n; t += NT) {
      const double x = vn[pos[t]];
      if (x > best || (x != x && best == best)) {
        best = x;
        bt = t;
      }
    }
    const unsigned key = wave_max_key(argmax_key<6>(best, lane));
    unsigned* redk = reinterpret_cast<unsigned*>(red);
    if (key != 0u && lane == argmax_key_index<6>(key)) {
      redk[wave] = key;
      redi[wave] = bt;
    } else if (key == 0u && lane == 0) {
      redk[wave] = 0u;
    }
    __syncthreads();
    unsigned kb = redk[0];
    int p = kb ? redi[0] : n;
#pragma unroll
    for (int w = 1; w < nwaves; ++w)
      if (redk[w] > kb) {
        kb = redk[w];
        p = redi[w];
      }
    const double b = kb ? vn[pos[p]] : -1.0;
    const double nrm = sqrt(b > 0.0 ? b : 0.0);
    if (j == 0) r00 = nrm;
    int stop;
    if (D.target >= 0) stop = (j >= D.target);
    else stop = !(r00 > 0.0) || !(nrm > tol * r00);  // NaN-safe
    if (p >= n) stop = 1;  // no admissible pivot (non-finite norms)
    if (j == 0 && tid == 0) stg(D.r00, r00);
    if (stop) break;  // uniform: every thread decided from the same slots
    // Householder reflector H = I - tau v v^H with v_0 = 1 mapping the pivot
    // column's trailing part y = [alpha; x] to beta e_1, beta = -e^{i arg alpha} |y|.
    if (wave == 0) {
      const int cp = pos[p];
      cplx* cj = D.A + ld * cp;
      double s = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) s += abs2(ldg(cj + i));
      s = wave_sum(s);
      const cplx alpha = ldg(cj + j);
      const double aa = sqrt(abs2(alpha));
      const double nr = sqrt(aa * aa + s);
      cplx beta, u0;
      double tau;
      if (nr == 0.0) {
        beta = mk(0, 0);
        u0 = mk(1, 0);
        tau = 0.0;
      } else {
        const cplx ph = aa > 0.0 ? mk(alpha.re / aa, alpha.im / aa) : mk(1, 0);
        beta = mk(-ph.re * nr, -ph.im * nr);
        u0 = alpha - beta;
        const double u0a = abs2(u0);
        tau = 2.0 / (1.0 + s / u0a);
      }
      for (int i = j + 1 + lane; i < m; i += 64) v[i] = cdiv(ldg(cj + i), u0);
      if (lane == 0) {
        v[j] = mk(1, 0);
        stg(cj + j, beta);
        s_tau = tau;
        pos[p] = pos[j];
        pos[j] = cp;
      }
    }
    __syncthreads();
    const double tau = s_tau;
    // apply to the columns at positions j+1..n-1, CB at a time per wavefront
    const int rows = m - j;
    if (rows <= R * 64) {
      for (int t0 = j + 1 + CB * wave; t0 < n; t0 += CB * nwaves)
        reflect_columns<R, CB>(D, j, pos + t0, min(CB, n - t0), v + j, tau, vn, lane);
    } else {
      for (int t = j + 1 + wave; t < n; t += nwaves) reflect_column_long(D, j, pos[t], v + j, tau, vn, lane);
    }
    __syncthreads();
  }
  const int k = j;
  for (int c = tid; c < n; c += NT) stg(D.perm + c, pos[c]);
  if (tid == 0) stg(D.rank, k);
  if (want_T) {
    // T = R11^{-1} R12 in place, one column per thread; the row sums are
    // unrolled so that their independent loads are in flight together
    for (int t = k + tid; t < n; t += NT) {
      cplx* col = D.A + ld * pos[t];
      for (int i = k - 1; i >= 0; --i) {
        cplx s = ldg(col + i), s2 = mk(0, 0);
        int l = i + 1;
#pragma unroll 4
        for (; l + 1 < k; l += 2) {
          const cplx r = ldg(D.A + i + ld * pos[l]), r2 = ldg(D.A + i + ld * pos[l + 1]);
          const cplx x = ldg(col + l), x2 = ldg(col + l + 1);
          s.re -= r.re * x.re - r.im * x.im;
          s.im -= r.re * x.im + r.im * x.re;
          s2.re -= r2.re * x2.re - r2.im * x2.im;
          s2.im -= r2.re * x2.im + r2.im * x2.re;
        }
        if (l < k) {
          const cplx r = ldg(D.A + i + ld * pos[l]);
          const cplx x = ldg(col + l);
          s.re -= r.re * x.re - r.im * x.im;
          s.im -= r.re * x.im + r.im * x.re;
        }
        stg(col + i, cdiv(s + s2, ldg(D.A + i + ld * pos[i])));
      }
    }
  }
  __syncthreads();
}

// One workgroup per matrix (queue == nullptr), or a persistent grid whose
// workgroups take matrices from a work queue: *queue counts the matrices
// handed out and must be zero at launch.  Every workgroup leaves the loop
// once the counter passes count.
template <int NT, int R, int CB>
__global__ __launch_bounds__(NT) void k_cpqr(const IdDesc* __restrict__ descs, int count, double tol, int want_T,
                                             int* queue) {
  extern __shared__ double lds[];
  if (queue == nullptr) {
    const IdDesc D = descs[blockIdx.x];
    cpqr_one<NT, R, CB>(D, tol, want_T, lds);
    return;
  }
  __shared__ int s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(queue, 1);
    __syncthreads();
    const int d = s_next;
    __syncthreads();
    if (d >= count) break;
    const IdDesc D = descs[d];
    cpqr_one<NT, R, CB>(D, tol, want_T, lds);
    __syncthreads();
  }
}


__global__ void k_build_interp(const InterpDesc* __restrict__ descs) {
  const InterpDesc D = descs[blockIdx.y];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= D.n) return;
  const int pc = D.perm[c];
  const long ldo = D.ldo;
  if (c < D.k) {
    const long idx = D.transpose ? (D.col0 + pc) + ldo * (D.row0 + c) : (D.row0 + c) + ldo * (D.col0 + pc);
    D.out[idx] = mk(1, 0);
  } else {
    const cplx* tc = D.A + (long)D.ld * pc;  // column c of T stays in place at perm[c]
    for (int r = 0; r < D.k; ++r) {
      const long idx = D.transpose ? (D.col0 + pc) + ldo * (D.row0 + r) : (D.row0 + r) + ldo * (D.col0 + pc);
      D.out[idx] = tc[r];
    }
  }
}

// Two-sided baseline: give the two IDs of each (box, half) the same rank
// max(k_row, k_col), so that the compressed diagonal blocks stay square.
__global__ void k_equalise_ranks(int npairs, const int* __restrict__ ia, const int* __restrict__ ib,
                                 IdDesc* descs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  IdDesc& a = descs[ia[i]];
  IdDesc& b = descs[ib[i]];
  const int ka = *a.rank, kb = *b.rank;
  const int k = ka > kb ? ka : kb;
  a.target = k;
  b.target = k;
}

size_t cpqr_lds_bytes(int mmax, int nmax) {
  return sizeof(double) * (size_t)nmax + sizeof(cplx) * (size_t)mmax + 16 * (sizeof(double) + sizeof(int)) +
         sizeof(int) * (size_t)nmax + 64;
}

// Variants: 256 threads (4 wavefronts, several workgroups per CU; CB = 4
// columns per wavefront) or 1024 threads (16 wavefronts for few, large
// matrices; CB = 2, or 1 with 8 register rows, to stay within 128
// registers); R = 4 or 8 register rows
// per lane by the tallest matrix.  persistent: queue-driven grid sized to the
// resident workgroups.
template <int NT, int R, int CB>
static void launch_cpqr_t(hipStream_t st, const IdDesc* descs, int count, size_t lds, double tol, int want_T,
                          int* queue) {
  if (!queue) {
    hipLaunchKernelGGL((k_cpqr<NT, R, CB>), dim3(count), dim3(NT), lds, st, descs, count, tol, want_T, nullptr);
    return;
  }
  int dev = 0, ncu = 0, per = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cpqr<NT, R, CB>, NT, lds));
  const int grid = std::max(1, std::min(count, ncu * std::max(per, 1)));
  hipLaunchKernelGGL((k_cpqr<NT, R, CB>), dim3(grid), dim3(NT), lds, st, descs, count, tol, want_T, queue);
}

void launch_cpqr(hipStream_t st, const IdDesc* descs, int count, int mmax, int nmax, double tol, int want_T,
                 const CpqrVariant& var, int* queue, bool resume) {
  if (count <= 0) return;
  if (var.qr) {
    launch_id_qr(st, descs, count, mmax, nmax, tol, want_T, resume);
    return;
  }
  const size_t lds = cpqr_lds_bytes(mmax, nmax);
  if (lds > 160 * 1024) throw std::runtime_error("proxy matrix too large for the ID kernel's LDS staging");

  int* q = var.persistent ? queue : nullptr;
  if (var.persistent) {
    if (!queue) throw std::invalid_argument("persistent ID launch without a queue counter");
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, queue, 1);
  }
  const bool tall = mmax > 256;
  if (var.threads == 1024) {
    if (tall) launch_cpqr_t<1024, 8, 1>(st, descs, count, lds, tol, want_T, q);
    else launch_cpqr_t<1024, 4, 2>(st, descs, count, lds, tol, want_T, q);
  } else {
    if (tall) launch_cpqr_t<256, 8, 4>(st, descs, count, lds, tol, want_T, q);
    else launch_cpqr_t<256, 4, 4>(st, descs, count, lds, tol, want_T, q);
  }
  HIPCHK(hipGetLastError());
}

CpqrVariant cpqr_default_variant(int count, int mmax, int nmax) {
  CpqrVariant v;
  v.threads = count >= 128 ? 256 : 1024;
  v.persistent = 0;
  // the two-stage kernels pay off when many matrices fill the chip; for a
  // few matrices the one-stage 1024-thread kernel is faster (measured: the
  // 512 leaf halves of the 32768-node star 1.6 against 2.6 ms, the 32
  // halves of its level 4 0.89 against 0.77 ms)
  v.qr = (count >= 128 && id_qr_eligible(mmax, nmax)) ? 1 : 0;
  return v;
}

void launch_build_interp(hipStream_t st, const InterpDesc* descs, int count, int nmax) {
  if (count <= 0 || nmax <= 0) return;
  hipLaunchKernelGGL(k_build_interp, dim3(cdiv_int(nmax, 128), count), dim3(128), 0, st, descs);
  HIPCHK(hipGetLastError());
}

void launch_equalise_ranks(hipStream_t st, int npairs, const int* ia, const int* ib, IdDesc* descs) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(k_equalise_ranks, dim3(cdiv_int(npairs, 128)), dim3(128), 0, st, npairs, ia, ib, descs);
  HIPCHK(hipGetLastError());
}

}  // namespace symhss

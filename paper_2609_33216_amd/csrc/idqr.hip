// Interpolative decomposition of proxy matrices (paper Section 4.1, the ID of
// each half of M_R, eq. low-rank_R) in two kernels, for matrices of at most
// 128 columns and 512 rows:
//
//  1. k_id_qr: unpivoted Householder QR of M (m x n) in place, in panels of
//     16 columns.  A panel is factored in registers; its reflectors are
//     accumulated in the compact form Q = I - V T V^H (T upper triangular,
//     from the Gram matrix of V), and the trailing columns are updated as
//     A := A - V (T^H (V^H A)) on the matrix cores (v_mfma_f64_16x16x4).
//     Each trailing column is read twice and written once per panel.
//  2. k_id_sq: column-pivoted Householder QR of the min(m, n) x n triangle R0
//     held entirely in registers (no memory traffic inside the pivot loop),
//     then T = R11^{-1} R12 from the packed R11 in LDS.
//
// Since M = Q0 R0 with Q0 unitary, every column norm and every inner product
// of columns of M equals that of R0: pivoted QR of R0 takes the same pivots
// as pivoted QR of M (in exact arithmetic), stops at the same rank under the
// rule |R_jj| <= tol |R_00| and gives the same T.  The outputs are those of
// k_cpqr: column t of R (or of T) in the memory of original column perm[t],
// rank, |R_00|.
#include <algorithm>

#include "kernels.hpp"

namespace symhss {

namespace {

typedef double qr_d4 __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 FP64 matrix-core step: A[i][k] from lane i + 16 k, B[k][j]
// from lane j + 16 k; item r of lane l accumulates D[4 r + l / 16][l % 16].
__device__ __forceinline__ qr_d4 mma(double a, double b, qr_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Sum over the 8 aligned lanes 8p .. 8p + 7 (every lane of the group
// receives the same value): quad exchanges, then the half-row mirror.
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);  // row_half_mirror: lane i <-> 7 - i of each 8
  return v;
}

// Householder reflector H = I - tau v v^H, v_0 = 1, mapping [alpha; x] (with
// s = |x|^2) to beta e_1, beta = -e^{i arg alpha} |[alpha; x]|; u0 is the
// divisor that turns x into v.  tau is real, so H is Hermitian and unitary.
struct Reflector {
  cplx beta, u0;
  double tau;
};
__device__ inline Reflector make_reflector(cplx alpha, double s) {
  Reflector R;
  const double aa = sqrt(abs2(alpha));
  const double nr = sqrt(aa * aa + s);
  if (nr == 0.0) {
    R.beta = mk(0, 0);
    R.u0 = mk(1, 0);
    R.tau = 0.0;
  } else {
    const cplx ph = aa > 0.0 ? mk(alpha.re / aa, alpha.im / aa) : mk(1, 0);
    R.beta = mk(-ph.re * nr, -ph.im * nr);
    R.u0 = alpha - R.beta;
    R.tau = 2.0 / (1.0 + s / abs2(R.u0));
  }
  return R;
}

constexpr int kQrNb = 16;   // panel width of the unpivoted QR
constexpr int kSqMax = 128;  // largest order held by the pivoted QR in registers
constexpr int kSqThreads = 1024;

}  // namespace

// Column jj = 4 Q + (owner wavefront) of a panel of k_id_qr.  Only the slot
// Q is a template argument: sixteen unrolled column steps of a 256-row panel
// take over 100 KB of code, more than the instruction cache holds.  Complex
// values are selected by component (a select of whole structures becomes a
// select of their addresses, which keeps the register array in memory).
__device__ __forceinline__ cplx csel(bool p, cplx x, cplx y) { return mk(p ? x.re : y.re, p ? x.im : y.im); }

template <int RPL, int Q>
__device__ __forceinline__ void qr_column(cplx (&a)[4][RPL], cplx (*vb)[64 * RPL], double* taus, cplx* Gs, int j0,
                                          int jj, int nb, int m, int lane, int wave) {
  const int j = j0 + jj;
  const int buf = jj & 1;
  if (wave == (jj & 3)) {
    cplx x = mk(0, 0);
#pragma unroll
    for (int r = 0; r < RPL; ++r) x = csel(lane + 64 * r == j, a[Q][r], x);
    const cplx alpha = mk(readlane_f64(x.re, j & 63), readlane_f64(x.im, j & 63));
    double s2 = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int row = lane + 64 * r;
      if (row > j) s2 += abs2(a[Q][r]);
    }
    s2 = wave_sum_dpp(s2);
    const Reflector H = make_reflector(alpha, s2);
    const cplx ru = cdiv(mk(1, 0), H.u0);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int row = lane + 64 * r;
      const cplx vx = a[Q][r] * ru;  // rows >= m hold zeros
      const bool below = row > j, diag = row == j;
      const cplx v = mk(below ? vx.re : (diag ? 1.0 : 0.0), below ? vx.im : 0.0);
      a[Q][r] = csel(diag, H.beta, csel(below, v, a[Q][r]));  // R above the diagonal stays
      vb[buf][row] = v;
    }
    if (lane == 0) taus[jj] = H.tau;
  }
  __syncthreads();
  const double tau = taus[jj];
  cplx v[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) v[r] = vb[buf][lane + 64 * r];
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    const int jq = wave + 4 * qq;
    if (jq > jj && jq < nb) {
      // a -= tau v (v^H a); v vanishes above row j
      cplx w = mk(0, 0);
#pragma unroll
      for (int r = 0; r < RPL; ++r) fma_conj_acc(w, v[r], a[qq][r]);
      w.re = wave_sum_dpp(w.re);
      w.im = wave_sum_dpp(w.im);
      const cplx tw = tau * w;
#pragma unroll
      for (int r = 0; r < RPL; ++r) fma_acc(a[qq][r], -v[r], tw);
    } else if (jq < jj) {
      // Gram entry v_jq^H v_jj: the stored reflector jq below its diagonal
      // meets v_jj, which vanishes above row j > j0 + jq
      cplx gsum = mk(0, 0);
#pragma unroll
      for (int r = 0; r < RPL; ++r) fma_conj_acc(gsum, a[qq][r], v[r]);
      gsum.re = wave_sum_dpp(gsum.re);
      gsum.im = wave_sum_dpp(gsum.im);
      if (lane == 0) Gs[jq * kQrNb + jj] = gsum;
    }
  }
}

// ---------------------------------------------------------------------------
// 1. Unpivoted blocked QR.  One workgroup of 256 threads per matrix; rows
// 0 .. 64 RPL - 1 (RPL rows per lane).  In a panel [j0, j0 + 16), wavefront w
// holds panel columns w, w + 4, w + 8, w + 12 in registers (lane l: rows
// l + 64 r).  Per column: the owner forms the reflector and stores it in its
// column (beta on the diagonal, v below), the other wavefronts apply it to
// their later columns and form the Gram entries v_a^H v_b of their earlier
// ones; one barrier per column (the reflector alternates between two LDS
// buffers).  Then T (LAPACK's forward accumulation, T(0:b, b) = -tau_b
// T(0:b, 0:b) V(:, 0:b)^H v_b) and the trailing update, 16 columns per
// wavefront task:
//   W = V^H A_t (16 x 16, contraction over the rows j0 .. m - 1),
//   X = T^H W, A_t -= V X,
// all three products on the matrix cores with complex entries as four real
// products.  The accumulator of W is laid out as the B operand of T^H W, and
// that of X as the A operand of (V X)^T, so neither leaves the registers.
template <int RPL>
__global__ __launch_bounds__(256) void k_id_qr(const IdDesc* __restrict__ descs) {
  __shared__ cplx vb[2][64 * RPL];
  __shared__ double taus[kQrNb];
  __shared__ cplx Gs[kQrNb * kQrNb];  // Gs[a * 16 + b] = v_a^H v_b, a < b
  __shared__ cplx Ts[kQrNb * kQrNb];  // Ts[r * 16 + c] = T[r][c]
  const IdDesc D = descs[blockIdx.x];
  const int m = D.m, n = D.n;
  const long ld = D.ld;
  cplx* __restrict__ A = D.A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lq = lane & 15, lk = lane >> 4;
  const int kmax = m < n ? m : n;

  for (int j0 = 0; j0 < kmax; j0 += kQrNb) {
    const int nb = min(kQrNb, n - j0);       // panel columns present
    const int nsteps = min(kQrNb, kmax - j0);  // reflectors of this panel
    cplx a[4][RPL];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jq = wave + 4 * q;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int row = lane + 64 * r;
        a[q][r] = mk(0, 0);
        if (jq < nb && row < m) a[q][r] = ldg(A + row + ld * (j0 + jq));
      }
    }
    for (int w4 = 0; w4 < 4; ++w4)
      if (w4 < nsteps) qr_column<RPL, 0>(a, vb, taus, Gs, j0, w4, nb, m, lane, wave);
    for (int w4 = 0; w4 < 4; ++w4)
      if (4 + w4 < nsteps) qr_column<RPL, 1>(a, vb, taus, Gs, j0, 4 + w4, nb, m, lane, wave);
    for (int w4 = 0; w4 < 4; ++w4)
      if (8 + w4 < nsteps) qr_column<RPL, 2>(a, vb, taus, Gs, j0, 8 + w4, nb, m, lane, wave);
    for (int w4 = 0; w4 < 4; ++w4)
      if (12 + w4 < nsteps) qr_column<RPL, 3>(a, vb, taus, Gs, j0, 12 + w4, nb, m, lane, wave);
    // the factored panel back to memory (rows j0 .. m - 1)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jq = wave + 4 * q;
      if (jq < nb) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int row = lane + 64 * r;
          if (row >= j0 && row < m) stg(A + row + ld * (j0 + jq), a[q][r]);
        }
      }
    }
    __syncthreads();
    if (wave == 0 && lane < kQrNb) {
      // row `lane` of T, column by column; absent reflectors give zero rows
      // and columns
      const int i = lane;
      for (int b = 0; b < kQrNb; ++b) {
        cplx tv = mk(0, 0);
        if (b < nsteps) {
          const double tb = taus[b];
          if (i < b) {
            cplx s = mk(0, 0);
            for (int l = i; l < b; ++l) fma_acc(s, Ts[i * kQrNb + l], Gs[l * kQrNb + b]);
            tv = mk(-tb * s.re, -tb * s.im);
          } else if (i == b) {
            tv = mk(tb, 0);
          }
        }
        Ts[i * kQrNb + b] = tv;
      }
    }
    __syncthreads();
    // V[rr][i] (rr counted from row j0): unit lower trapezoid of the panel
    auto vop = [&](int rr, int i) -> cplx {
      if (i >= nsteps || rr < i || j0 + rr >= m) return mk(0, 0);
      if (rr == i) return mk(1, 0);
      return ldg(A + (j0 + rr) + ld * (j0 + i));
    };
    const int K = m - j0;
    const int c_first = j0 + kQrNb;
    const int ntile = n > c_first ? (n - c_first + 15) / 16 : 0;
    for (int ct = wave; ct < ntile; ct += 4) {
      const int c0 = c_first + 16 * ct;
      const bool colok = c0 + lq < n;
      // W = V^H A_t: lane (lq, lk) supplies rows g + 4 lk + s in step s
      qr_d4 wr = {0, 0, 0, 0}, wi = {0, 0, 0, 0};
      cplx vv[4], at[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int rr = 4 * lk + s;
        vv[s] = vop(rr, lq);
        at[s] = mk(0, 0);
        if (colok && j0 + rr < m) at[s] = ldg(A + (j0 + rr) + ld * (c0 + lq));
      }
      for (int g = 0; g < K; g += 16) {
        // the next group's operands are loaded while this one is multiplied
        cplx vn[4], an[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int rr = g + 16 + 4 * lk + s;
          vn[s] = vop(rr, lq);
          an[s] = mk(0, 0);
          if (colok && j0 + rr < m) an[s] = ldg(A + (j0 + rr) + ld * (c0 + lq));
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          wr = mma(vv[s].re, at[s].re, wr);
          wr = mma(vv[s].im, at[s].im, wr);
          wi = mma(vv[s].re, at[s].im, wi);
          wi = mma(-vv[s].im, at[s].re, wi);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          vv[s] = vn[s];
          at[s] = an[s];
        }
      }
      // X = T^H W: step s contracts k = 4 s + lk; W[k][lq] is item s of this lane
      qr_d4 xr = {0, 0, 0, 0}, xi = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const cplx tv = Ts[(4 * s + lk) * kQrNb + lq];  // T[k][i], i = lq
        xr = mma(tv.re, wr[s], xr);
        xr = mma(tv.im, wi[s], xr);
        xi = mma(tv.re, wi[s], xi);
        xi = mma(-tv.im, wr[s], xi);
      }
      // A_t -= V X as (V X)^T = X^T V^T per 16-row block: X[k][lq] (k =
      // 4 s + lk) is item s of this lane; item r of the result is row
      // g + lq, column c0 + 4 r + lk of the tile
      cplx vu[4], cu[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int col = c0 + 4 * s + lk;
        vu[s] = vop(lq, 4 * s + lk);
        cu[s] = mk(0, 0);
        if (j0 + lq < m && col < n) cu[s] = ldg(A + (j0 + lq) + ld * col);
      }
      for (int g = 0; g < K; g += 16) {
        cplx vn[4], cn[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int rown = j0 + g + 16 + lq, col = c0 + 4 * s + lk;
          vn[s] = vop(g + 16 + lq, 4 * s + lk);
          cn[s] = mk(0, 0);
          if (rown < m && col < n) cn[s] = ldg(A + rown + ld * col);
        }
        qr_d4 dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          dr = mma(xr[s], vu[s].re, dr);
          dr = mma(-xi[s], vu[s].im, dr);
          di = mma(xr[s], vu[s].im, di);
          di = mma(xi[s], vu[s].re, di);
        }
        const int row = j0 + g + lq;
        if (row < m) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int col = c0 + 4 * r + lk;
            if (col < n) stg(A + row + ld * col, mk(cu[r].re - dr[r], cu[r].im - di[r]));
          }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          vu[s] = vn[s];
          cu[s] = cn[s];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 2. Pivoted QR of the triangle in registers.  1024 threads: the 8 lanes
// 8c .. 8c + 7 hold column c, lane 8c + g its rows 16 g .. 16 g + 15 (the
// whole 128 x 128 matrix in 64 registers per lane).  Column interchanges are
// logical: each column carries its position; the pivot is the position >= j
// of largest trailing norm (norms recomputed exactly after every step; among
// norms equal to about 2^-12 relative, the lowest position).  Per step: the
// wavefronts' best keys meet in LDS (barrier), the wavefront holding the
// pivot forms its reflector in LDS (barrier), every other column applies it.
// Input: the upper triangle of rows 0 .. min(m, n) - 1 (the strictly lower
// part, which holds the QR's reflectors, is read as zero) or, when resuming
// (target >= 0 and rank > 0), the state a previous pass left.  Then
// T = R11^{-1} R12 by backward substitution in LDS, eight threads per column.
constexpr int kSqWaves = kSqThreads / 64;

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__global__ __launch_bounds__(kSqThreads) void k_id_sq(const IdDesc* __restrict__ descs, double tol, int want_T) {
  extern __shared__ double sqlds[];
  __shared__ cplx vsh[kSqMax];  // the step's reflector
  __shared__ unsigned skey[kSqWaves];
  __shared__ double svn[kSqWaves];
  __shared__ double stau;
  __shared__ int scp;
  __shared__ int posl[kSqMax];  // column at each position (for T)
  const IdDesc D = descs[blockIdx.x];
  const int n = D.n, m = D.m < D.n ? D.m : D.n;
  const long ld = D.ld;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = t & 7, c = t >> 3;
  constexpr int nw = kSqWaves;

  const int j0 = (D.target >= 0) ? ldg(D.rank) : 0;
  if (j0 > 0)
    for (int q = t; q < n; q += kSqThreads) posl[ldg(D.perm + q)] = q;  // inverse of perm, used once
  __syncthreads();
  const bool ok = c < n;
  int pos = ok ? (j0 > 0 ? posl[c] : c) : (1 << 20);
  bool done = !ok || pos < j0;
  cplx a[16];
  double vn;
  {
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = 16 * g + e;
      a[e] = mk(0, 0);
      if (ok && row < m && (j0 > 0 || row <= c)) a[e] = ldg(D.A + row + ld * c);
      if (row >= j0) s += abs2(a[e]);
    }
    vn = group8_sum(s);
  }
  double r00 = (j0 > 0) ? ldg(D.r00) : 0.0;
  const int kmax = m < n ? m : n;
  int j = j0;
  for (; j < kmax; ++j) {
    // the wavefronts' best columns
    {
      const unsigned key = done ? 0u : argmax_key<7>(vn, pos);
      const unsigned wk = wave_max_key(key);
      const unsigned long long bal = __ballot(wk != 0u && key == wk);
      const int bl = bal ? __ffsll((long long)bal) - 1 : 0;
      const double bv = readlane_f64(vn, bl);
      if (lane == 0) {
        skey[wave] = wk;
        svn[wave] = bv;
      }
    }
    __syncthreads();
    unsigned K = 0u;
    int ww = 0;
#pragma unroll
    for (int w = 0; w < nw; ++w) {
      const unsigned kw = skey[w];
      if (kw > K) {
        K = kw;
        ww = w;
      }
    }
    K = (unsigned)uniform((int)K);
    ww = uniform(ww);
    if (K == 0u) break;  // no admissible pivot (non-finite norms)
    const double bvn = svn[ww];
    const double nrm = sqrt(bvn > 0.0 ? bvn : 0.0);
    if (j == 0) r00 = nrm;
    const int stop = (D.target >= 0) ? (j >= D.target) : (!(r00 > 0.0) || !(nrm > tol * r00));  // NaN-safe
    if (uniform(stop)) break;
    const int p = argmax_key_index<7>(K);
    if (wave == ww) {
      // the pivot column's reflector
      const bool mine = !done && pos == p;
      const int base = __ffsll((long long)__ballot(mine)) - 1;
      const int je = j & 15;
      cplx xj = a[0];
#pragma unroll
      for (int e = 1; e < 16; ++e)
        if (je == e) xj = a[e];
      const cplx alpha = mk(readlane_f64(xj.re, base + (j >> 4)), readlane_f64(xj.im, base + (j >> 4)));
      double s = 0.0;
      if (mine) {
#pragma unroll
        for (int e = 0; e < 16; ++e)
          if (16 * g + e > j) s += abs2(a[e]);
      }
      s = wave_sum_dpp(s);
      const Reflector H = make_reflector(alpha, s);
      if (mine) {
        const cplx ru = cdiv(mk(1, 0), H.u0);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int row = 16 * g + e;
          const cplx vx = a[e] * ru;
          const bool below = row > j, diag = row == j;
          vsh[row] = mk(below ? vx.re : (diag ? 1.0 : 0.0), below ? vx.im : 0.0);
          a[e] = mk(below ? 0.0 : (diag ? H.beta.re : a[e].re), below ? 0.0 : (diag ? H.beta.im : a[e].im));
        }
        done = true;
      }
      if (lane == 0) {
        stau = H.tau;
        scp = 8 * wave + (base >> 3);
      }
    }
    __syncthreads();
    if (pos == j) pos = p;
    if (c == scp) pos = j;
    if (!done) {
      // the reflector is read from LDS twice (products, then the update), so
      // that only the column stays in registers
      const double tau = stau;
      const cplx* vr = vsh + 16 * g;
      cplx w = mk(0, 0);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        fma_conj_acc(w, vr[e], a[e]);
        if ((e & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the loads in flight (registers)
      }
      w.re = group8_sum(w.re);
      w.im = group8_sum(w.im);
      const cplx tw = tau * w;
      double s = 0.0;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        fma_acc(a[e], -vr[e], tw);
        if (16 * g + e > j) s += abs2(a[e]);
        if ((e & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
      vn = group8_sum(s);
    }
  }
  const int k = j;
  if (t == 0) {
    stg(D.rank, k);
    if (j0 == 0) stg(D.r00, r00);
  }
  if (ok && g == 0) stg(D.perm + pos, c);
  if (!want_T) {
    // the state, for a pass that resumes
    if (ok) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = 16 * g + e;
        if (row < m) stg(D.A + row + ld * c, a[e]);
      }
    }
    return;
  }
  // LDS: R11 packed by columns (column p, rows 0 .. p, at p (p + 1) / 2),
  // then the reciprocals of its diagonal, then R12 by position (column
  // t >= k, rows 0 .. k - 1, at (t - k) k)
  __syncthreads();  // posl is rewritten below
  const int nt = n - k;
  cplx* Rp = reinterpret_cast<cplx*>(sqlds);
  cplx* rinv = Rp + k * (k + 1) / 2;
  cplx* Bt = rinv + k;
  if (ok) {
    if (g == 0) posl[pos] = c;
    if (pos < k) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = 16 * g + e;
        if (row <= pos) Rp[pos * (pos + 1) / 2 + row] = a[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = 16 * g + e;
        if (row < k) Bt[(pos - k) * k + row] = a[e];
      }
    }
  }
  __syncthreads();
  for (int i = t; i < k; i += kSqThreads) rinv[i] = cdiv(mk(1, 0), Rp[i * (i + 1) / 2 + i]);
  __syncthreads();
  // column q of T: the 8 lanes 8q .. 8q + 7; lane g owns rows g, g + 8, ...
  // (only it reads or writes them), and x_i goes from the owner of row i to
  // the group by a lane exchange
  const int src0 = lane & ~7;
  for (int q0 = 0; q0 < nt; q0 += kSqThreads / 8) {
    const int q = q0 + (t >> 3);
    const bool qok = q < nt;
    cplx* b = Bt + (long)(qok ? q : 0) * k;
    for (int i = k - 1; i >= 0; --i) {
      cplx x = mk(0, 0);
      if (qok && g == (i & 7)) {
        x = b[i] * rinv[i];
        b[i] = x;
      }
      x.re = __shfl(x.re, src0 + (i & 7));
      x.im = __shfl(x.im, src0 + (i & 7));
      if (qok) {
        const cplx* ri = Rp + i * (i + 1) / 2;
        for (int l = g; l < i; l += 8) fma_acc(b[l], -ri[l], x);
      }
    }
  }
  __syncthreads();
  for (int e = t; e < nt * k; e += kSqThreads) {
    const int q = e / k, i = e % k;
    stg(D.A + i + ld * posl[k + q], Bt[e]);
  }
}

bool id_qr_eligible(int mmax, int nmax) { return nmax <= kSqMax && mmax <= 512; }

void launch_id_qr(hipStream_t st, const IdDesc* descs, int count, int mmax, int nmax, double tol, int want_T,
                  bool resume) {
  if (count <= 0) return;
  if (!id_qr_eligible(mmax, nmax)) throw std::invalid_argument("matrix too large for the two-stage ID kernels");
  if (!resume) {
    if (mmax <= 128) hipLaunchKernelGGL(k_id_qr<2>, dim3(count), dim3(256), 0, st, descs);
    else if (mmax <= 256) hipLaunchKernelGGL(k_id_qr<4>, dim3(count), dim3(256), 0, st, descs);
    else hipLaunchKernelGGL(k_id_qr<8>, dim3(count), dim3(256), 0, st, descs);
    HIPCHK(hipGetLastError());
  }
  // dynamic LDS for T: R11 packed, its reciprocal diagonal and R12, for the
  // largest rank the launch can reach
  const int r = std::min(nmax, kSqMax);
  long ent = 0;
  for (int k = 0; k <= r; ++k) ent = std::max<long>(ent, (long)k * (k + 1) / 2 + k + (long)k * (nmax - k));
  const int lds = (int)(ent * sizeof(cplx));
  hipLaunchKernelGGL(k_id_sq, dim3(count), dim3(kSqThreads), lds, st, descs, tol, want_T);
  HIPCHK(hipGetLastError());
}

}  // namespace symhss

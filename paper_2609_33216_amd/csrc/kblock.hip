// Kernel-block generation for the Muller-like 2x2 Nystrom system, FP64.
//
// Entry between observation point o and source point s (paper Section 3.1,
// eq. symmetric_muller / eq. block_A), with d = x_o - x_s, r = |d|,
// omega = w_o w_s (row-scaled) or w_s (unscaled, eq. naive_muller):
//   A11 = -omega (i/4) (eps0^2 H0(k0 r) - eps1^2 H0(k1 r))
//   A12 =  omega (i/4) (eps0 k0 H1(k0 r) - eps1 k1 H1(k1 r)) (d.nu_s)/r
//   A21 = -omega (i/4) (eps0 k0 H1(k0 r) - eps1 k1 H1(k1 r)) (d.nu_o)/r
//   A22 = -omega (N_k0 - N_k1),
//   N_k0 - N_k1 = (i/4) [ dH1 (nu_o.nu_s / r - 2c / r^3) + dH0 c / r^2 ],
//   c = (d.nu_o)(d.nu_s), dH1 = k0 H1(k0 r) - k1 H1(k1 r), dH0 = k0^2 H0(k0 r) - k1^2 H0(k1 r).
// k H1(k r) = k J1 + i (k Y1reg(k r) - 2/(pi r)): the 2/(pi r) poles of the
// two wavenumbers are combined analytically, so dH1 carries no cancellation.
// On the diagonal (o = s, a boundary node) the one-point corrected values
// and the free terms -/+ (eps0 + eps1) w / 2 (or 1/2, unscaled) apply.
//
// The PMCHWT system (eq. symmetric_pmchwt / naive_pmchwt) combines the same
// kernels with other weights and no free terms:
//   A11 = -omega (eps0 G_k0 + eps1 G_k1),  A12 = omega (D_k0 + D_k1),
//   A21 = omega (D*_k0 + D*_k1),           A22 = -omega (N_k0/eps0 + N_k1/eps1),
// and the Burton-Miller system (eq. bm, alpha = i/k0, columns in [q; u]):
//   A11 = -omega eps0 (G_k0 + alpha D*_k0) - alpha eps0 f,  A12 = omega (D_k0 + alpha N_k0) - f,
//   A21 = -omega eps1 G_k1,                                 A22 = omega D_k1 + f,
// f = w/2 (row-scaled) or 1/2 on the diagonal.  Both need the individual,
// hypersingular N_k, whose one-point corrected diagonal is
//   -pi/(6 w^2) + kappa^2/(24 pi) + i k^2/8 - (k^2/4pi)(ln(k/2) + gamma - 1/2 + ln(w/2pi))
// (zeta(2) removes the trapezoidal rule's h^-1 term of the 1/t^2 part; the
// rule then converges at first order, as Section 3.1 states for N_k).
//
// One thread evaluates one point pair and writes its (up to) four entries;
// the Hankel functions of both wavenumbers are shared by the four.
#include "kernels.hpp"
#include "bessel.hpp"

namespace symhss {

// The Bessel evaluation is kept out of line: inlined twice (one per
// wavenumber) the compiler interleaves the two and the register count
// doubles, costing occupancy.
__device__ __noinline__ JY01 jy01_call(double z) { return jy01(z); }

__device__ inline void muller_pair(const PointsDev& P, const MediumDev& md, int io, int is,
                                   cplx e[4]) {
  const double e0 = md.eps0, e1 = md.eps1;
  const double wo = P.w[io], ws = P.w[is];
  const double om = md.row_scaled ? wo * ws : ws;
  if (io == is && io < P.n_boundary) {
    const double ell = log(wo * (0.5 / kPi));
    // G~_k = i/4 - (ln(k/2) + gamma + ell) / (2 pi)
    const double g0r = -(md.g0c + ell) * (0.5 / kPi);
    const double g1r = -(md.g1c + ell) * (0.5 / kPi);
    const double s_re = e0 * e0 * g0r - e1 * e1 * g1r;
    const double s_im = (e0 * e0 - e1 * e1) * 0.25;
    e[0] = mk(-om * s_re, -om * s_im);
    const double dd = (e0 - e1) * (-P.kappa[io] * (0.25 / kPi));
    const double fr = 0.5 * (e0 + e1) * (md.row_scaled ? wo : 1.0);
    e[1] = mk(om * dd - fr, 0.0);
    e[2] = mk(om * dd + fr, 0.0);
    const double nd_re = md.nd_re - md.delta * (0.25 / kPi) * ell;
    e[3] = mk(-om * nd_re, -om * md.nd_im);
    return;
  }
  const double dx = P.x[io] - P.x[is];
  const double dy = P.y[io] - P.y[is];
  const double r = sqrt(dx * dx + dy * dy);
  const double invr = 1.0 / r;
  const double dno = dx * P.nx[io] + dy * P.ny[io];
  const double dns = dx * P.nx[is] + dy * P.ny[is];
  const double nn = P.nx[io] * P.nx[is] + P.ny[io] * P.ny[is];
  const JY01 a = jy01_call(md.k0 * r);
  const JY01 b = jy01_call(md.k1 * r);
  const double k0 = md.k0, k1 = md.k1;
  const double pole = kTwoOverPi * invr;  // 2/(pi r)
  // A11: -(i/4) (eps0^2 H0a - eps1^2 H0b) * om
  {
    const double sr = e0 * e0 * a.j0 - e1 * e1 * b.j0;
    const double si = e0 * e0 * a.y0 - e1 * e1 * b.y0;
    // (i/4)(sr + i si) = (-si/4, sr/4)
    e[0] = mk(om * 0.25 * si, -om * 0.25 * sr);
  }
  // A12, A21
  {
    const double dr_ = e0 * k0 * a.j1 - e1 * k1 * b.j1;
    const double di_ = e0 * k0 * a.y1r - e1 * k1 * b.y1r - (e0 - e1) * pole;
    const double ire = -0.25 * di_, iim = 0.25 * dr_;  // (i/4)(dr + i di)
    const double f12 = om * dns * invr;
    const double f21 = -om * dno * invr;
    e[1] = mk(ire * f12, iim * f12);
    e[2] = mk(ire * f21, iim * f21);
  }
  // A22
  {
    const double h1r = k0 * a.j1 - k1 * b.j1;
    const double h1i = k0 * a.y1r - k1 * b.y1r;
    const double h0r = k0 * k0 * a.j0 - k1 * k1 * b.j0;
    const double h0i = k0 * k0 * a.y0 - k1 * k1 * b.y0;
    const double c = dno * dns;
    const double invr2 = invr * invr;
    const double f1 = nn * invr - 2.0 * c * invr2 * invr;
    const double f0 = c * invr2;
    const double sr = h1r * f1 + h0r * f0;
    const double si = h1i * f1 + h0i * f0;
    // -(om) (i/4)(sr + i si) = -om (-si/4, sr/4)
    e[3] = mk(om * 0.25 * si, -om * 0.25 * sr);
  }
}

// Hypersingular N_k diagonal: the k-independent part and the per-k part.
__device__ inline double n_hyp_diag(double w, double kappa) {
  return -kPi / (6.0 * w * w) + kappa * kappa * (1.0 / (24.0 * kPi));
}

__device__ inline void pmchwt_pair(const PointsDev& P, const MediumDev& md, int io, int is, cplx e[4]) {
  const double e0 = md.eps0, e1 = md.eps1, i0 = md.ie0, i1 = md.ie1;
  const double wo = P.w[io], ws = P.w[is];
  const double om = md.row_scaled ? wo * ws : ws;
  if (io == is && io < P.n_boundary) {
    const double ell = log(wo * (0.5 / kPi));
    const double g0r = -(md.g0c + ell) * (0.5 / kPi);
    const double g1r = -(md.g1c + ell) * (0.5 / kPi);
    e[0] = mk(-om * (e0 * g0r + e1 * g1r), -om * ((e0 + e1) * 0.25));
    const double dd = -P.kappa[io] * (0.25 / kPi);
    e[1] = mk(om * (dd + dd), 0.0);
    e[2] = e[1];
    const double hyp = n_hyp_diag(wo, P.kappa[io]);
    const double n0r = hyp + md.n0_re - md.k0 * md.k0 * (0.25 / kPi) * ell;
    const double n1r = hyp + md.n1_re - md.k1 * md.k1 * (0.25 / kPi) * ell;
    e[3] = mk(-om * (i0 * n0r + i1 * n1r), -om * (i0 * md.n0_im + i1 * md.n1_im));
    return;
  }
  const double dx = P.x[io] - P.x[is];
  const double dy = P.y[io] - P.y[is];
  const double r = sqrt(dx * dx + dy * dy);
  const double invr = 1.0 / r;
  const double dno = dx * P.nx[io] + dy * P.ny[io];
  const double dns = dx * P.nx[is] + dy * P.ny[is];
  const double nn = P.nx[io] * P.nx[is] + P.ny[io] * P.ny[is];
  const JY01 a = jy01_call(md.k0 * r);
  const JY01 b = jy01_call(md.k1 * r);
  const double k0 = md.k0, k1 = md.k1;
  const double pole = kTwoOverPi * invr;
  {
    const double sr = e0 * a.j0 + e1 * b.j0;
    const double si = e0 * a.y0 + e1 * b.y0;
    e[0] = mk(om * 0.25 * si, -om * 0.25 * sr);
  }
  {
    const double dr_ = k0 * a.j1 + k1 * b.j1;
    const double di_ = k0 * a.y1r + k1 * b.y1r - 2.0 * pole;
    const double ire = -0.25 * di_, iim = 0.25 * dr_;
    const double f12 = om * dns * invr;
    const double f21 = -om * dno * invr;
    e[1] = mk(ire * f12, iim * f12);
    e[2] = mk(ire * f21, iim * f21);
  }
  {
    const double h1r = i0 * k0 * a.j1 + i1 * k1 * b.j1;
    const double h1i = i0 * k0 * a.y1r + i1 * k1 * b.y1r - (i0 + i1) * pole;
    const double h0r = i0 * k0 * k0 * a.j0 + i1 * k1 * k1 * b.j0;
    const double h0i = i0 * k0 * k0 * a.y0 + i1 * k1 * k1 * b.y0;
    const double c = dno * dns;
    const double invr2 = invr * invr;
    const double f1 = nn * invr - 2.0 * c * invr2 * invr;
    const double f0 = c * invr2;
    const double sr = h1r * f1 + h0r * f0;
    const double si = h1i * f1 + h0i * f0;
    e[3] = mk(om * 0.25 * si, -om * 0.25 * sr);
  }
}

// (i/4) (re + i im)
__device__ inline cplx i4(double re, double im) { return mk(-0.25 * im, 0.25 * re); }

__device__ inline void bm_pair(const PointsDev& P, const MediumDev& md, int io, int is, cplx e[4]) {
  const double e0 = md.eps0, e1 = md.eps1;
  const cplx al = mk(md.al_re, md.al_im);
  const double wo = P.w[io], ws = P.w[is];
  const double om = md.row_scaled ? wo * ws : ws;
  if (io == is && io < P.n_boundary) {
    const double ell = log(wo * (0.5 / kPi));
    const cplx g0 = mk(-(md.g0c + ell) * (0.5 / kPi), 0.25);
    const cplx g1 = mk(-(md.g1c + ell) * (0.5 / kPi), 0.25);
    const double dd = -P.kappa[io] * (0.25 / kPi);
    const cplx n0 = mk(n_hyp_diag(wo, P.kappa[io]) + md.n0_re - md.k0 * md.k0 * (0.25 / kPi) * ell, md.n0_im);
    const double f = 0.5 * (md.row_scaled ? wo : 1.0);
    e[0] = (-e0 * om) * (g0 + dd * al) - (e0 * f) * al;
    e[1] = om * (mk(dd, 0.0) + al * n0) - mk(f, 0.0);
    e[2] = (-e1 * om) * g1;
    e[3] = mk(om * dd + f, 0.0);
    return;
  }
  const double dx = P.x[io] - P.x[is];
  const double dy = P.y[io] - P.y[is];
  const double r = sqrt(dx * dx + dy * dy);
  const double invr = 1.0 / r;
  const double dno = dx * P.nx[io] + dy * P.ny[io];
  const double dns = dx * P.nx[is] + dy * P.ny[is];
  const double nn = P.nx[io] * P.nx[is] + P.ny[io] * P.ny[is];
  const JY01 a = jy01_call(md.k0 * r);
  const JY01 b = jy01_call(md.k1 * r);
  const double k0 = md.k0, k1 = md.k1;
  const double pole = kTwoOverPi * invr;
  // k H1(k r) for both wavenumbers, k^2 H0(k0 r)
  const double h1ar = k0 * a.j1, h1ai = k0 * a.y1r - pole;
  const double h1br = k1 * b.j1, h1bi = k1 * b.y1r - pole;
  const cplx G0 = i4(a.j0, a.y0);
  const cplx G1 = i4(b.j0, b.y0);
  const cplx Dy0 = (dns * invr) * i4(h1ar, h1ai);
  const cplx Dx0 = (-dno * invr) * i4(h1ar, h1ai);
  const cplx Dy1 = (dns * invr) * i4(h1br, h1bi);
  const double c = dno * dns;
  const double invr2 = invr * invr;
  const double f1 = nn * invr - 2.0 * c * invr2 * invr;
  const double f0 = c * invr2;
  const cplx N0 = i4(h1ar * f1 + k0 * k0 * a.j0 * f0, h1ai * f1 + k0 * k0 * a.y0 * f0);
  e[0] = (-e0 * om) * (G0 + al * Dx0);
  e[1] = om * (Dy0 + al * N0);
  e[2] = (-e1 * om) * G1;
  e[3] = om * Dy1;
}

template <int EQ>
__device__ inline void system_pair(const PointsDev& P, const MediumDev& md, int io, int is, cplx e[4]) {
  if constexpr (EQ == kEqMuller) muller_pair(P, md, io, is, e);
  else if constexpr (EQ == kEqPmchwt) pmchwt_pair(P, md, io, is, e);
  else bm_pair(P, md, io, is, e);
}

template <int EQ>
__global__ __launch_bounds__(256) void k_kblock(PointsDev P, const MediumDev* __restrict__ media,
                                                const KJob* __restrict__ jobs,
                                                const KTile* __restrict__ tiles,
                                                const int* __restrict__ rpt, const int* __restrict__ rmap1,
                                                const int* __restrict__ rmap2, const int* __restrict__ cpt,
                                                const int* __restrict__ cmap1, const int* __restrict__ cmap2) {
  const KTile t = tiles[blockIdx.x];
  const KJob J = jobs[t.job];
  const MediumDev md = media[J.med];
  const int a = t.r0 + (threadIdx.x & 63);
  const int slot = threadIdx.x >> 6;
  if (a >= J.nr) return;
  const int ra = rpt[J.roff + a];
  const int o1 = rmap1[J.roff + a];
  const int o2 = rmap2[J.roff + a];
  const long ld = J.ld;
#pragma unroll 1
  for (int cc = slot; cc < 16; cc += 4) {
    const int b = t.c0 + cc;
    if (b >= J.nc) break;
    const int cb = cpt[J.coff + b];
    const int c1 = cmap1[J.coff + b];
    const int c2 = cmap2[J.coff + b];
    cplx e[4];
    system_pair<EQ>(P, md, ra, cb, e);
    if (J.mode != 2) {
      if (o1 >= 0 && c1 >= 0) J.out[o1 + ld * c1] = e[0];
      if (o1 >= 0 && c2 >= 0) J.out[o1 + ld * c2] = e[1];
      if (o2 >= 0 && c1 >= 0) J.out[o2 + ld * c1] = e[2];
      if (o2 >= 0 && c2 >= 0) J.out[o2 + ld * c2] = e[3];
    }
    if (J.mode != 0) {
      // entry (eq e at o, unknown t at s) = entry (eq t at s, unknown e at o)
      if (o1 >= 0 && c1 >= 0) J.out[c1 + ld * o1] = e[0];
      if (o1 >= 0 && c2 >= 0) J.out[c2 + ld * o1] = e[1];
      if (o2 >= 0 && c1 >= 0) J.out[c1 + ld * o2] = e[2];
      if (o2 >= 0 && c2 >= 0) J.out[c2 + ld * o2] = e[3];
    }
  }
}

// Nystrom geometry (paper Section 3.1): nu = (x2', -x1')/|x'| (into the
// exterior for a counter-clockwise curve), kappa = (x1' x2'' - x2' x1'')/|x'|^3,
// w = |x'| 2 pi / N.  Inputs are N x 2 interleaved.
__global__ void k_geometry(int n, const double* __restrict__ xin, const double* __restrict__ dxin,
                           const double* __restrict__ ddxin, double* px, double* py, double* nx, double* ny,
                           double* w, double* kappa) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d0 = dxin[2 * i], d1 = dxin[2 * i + 1];
  const double s = sqrt(d0 * d0 + d1 * d1);
  px[i] = xin[2 * i];
  py[i] = xin[2 * i + 1];
  nx[i] = d1 / s;
  ny[i] = -d0 / s;
  kappa[i] = (d0 * ddxin[2 * i + 1] - d1 * ddxin[2 * i]) / (s * s * s);
  w[i] = s * (2.0 * kPi / n);
}

// Plane-wave right-hand side: u_in = exp(i k0 d.x), q_in = i k0 (d.nu) u_in;
// Muller-like b = [-eps0 W u_in; W q_in] (row-scaled) or [-eps0 u_in; q_in],
// PMCHWT [-W u_in; W q_in / eps0], Burton-Miller [-(u_in + alpha q_in); 0].
// Right-hand side rows of node i from the incident trace u_in and its normal
// derivative q_in (eq. symmetric_muller / naive_muller, naive_pmchwt, bm);
// sc = w_i for the row-scaled systems, 1 otherwise.
__device__ inline void incident_rhs(const MediumDev& md, double sc, cplx uin, cplx qin, cplx& b1, cplx& b2) {
  if (md.eq == kEqPmchwt) {
    b1 = (-sc) * uin;
    b2 = (sc * md.ie0) * qin;
  } else if (md.eq == kEqBurtonMiller) {
    b1 = (-sc) * (uin + mk(md.al_re, md.al_im) * qin);
    b2 = mk(0.0, 0.0);
  } else {
    b1 = (-md.eps0 * sc) * uin;
    b2 = sc * qin;
  }
}

// u_in = exp(i k0 d.x), q_in = i k0 (d.nu) u_in at node i.
__device__ inline void plane_wave_at(const PointsDev& P, const MediumDev& md, double ca, double sa, int i,
                                     cplx& uin, cplx& qin) {
  const double ph = md.k0 * (ca * P.x[i] + sa * P.y[i]);
  double s, c;
  sincos(ph, &s, &c);
  const double dn = md.k0 * (ca * P.nx[i] + sa * P.ny[i]);
  uin = mk(c, s);
  qin = mk(-dn * s, dn * c);
}

__global__ void k_rhs_plane(int n, PointsDev P, MediumDev md, double ca, double sa, cplx* b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cplx uin, qin;
  plane_wave_at(P, md, ca, sa, i, uin, qin);
  incident_rhs(md, md.row_scaled ? P.w[i] : 1.0, uin, qin, b[i], b[n + i]);
}

__global__ void k_plane_incident(int n, PointsDev P, MediumDev md, double ca, double sa, cplx* uin, cplx* qin) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  plane_wave_at(P, md, ca, sa, i, uin[i], qin[i]);
}

// Column c of the right-hand sides: b[c ldb + (i, n + i)] from the traces
// uin[c ldi + i], qin[c ldi + i].
__global__ void k_rhs_incident(int n, PointsDev P, MediumDev md, const cplx* __restrict__ uin,
                               const cplx* __restrict__ qin, int ldi, cplx* __restrict__ b, int ldb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t c = blockIdx.y;
  cplx* bc = b + c * ldb;
  incident_rhs(md, md.row_scaled ? P.w[i] : 1.0, uin[c * ldi + i], qin[c * ldi + i], bc[i], bc[n + i]);
}

// Unknowns [q; u] of one boundary (column c at x + c ldx) -> the traces q, u.
__global__ void k_split_traces(int n, const cplx* __restrict__ x, int ldx, cplx* __restrict__ q,
                               cplx* __restrict__ u, int ldo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t c = blockIdx.y;
  q[c * ldo + i] = x[c * ldx + i];
  u[c * ldo + i] = x[c * ldx + n + i];
}

__global__ void k_bessel(int n, const double* __restrict__ z, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const JY01 r = jy01(z[i]);
  out[5 * i + 0] = r.j0;
  out[5 * i + 1] = r.y0;
  out[5 * i + 2] = r.j1;
  out[5 * i + 3] = r.y1;
  out[5 * i + 4] = r.y1r;
}

// Direct FP64 product y = A x without storing A: one thread per row of the
// 2N x 2N system, summing over all source nodes.
template <int EQ>
__global__ __launch_bounds__(256) void k_matvec_direct(PointsDev P, MediumDev md, const cplx* __restrict__ x,
                                                       cplx* __restrict__ y) {
  const int n = P.n_boundary;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cplx y1 = mk(0, 0), y2 = mk(0, 0);
  for (int j = 0; j < n; ++j) {
    cplx e[4];
    system_pair<EQ>(P, md, i, j, e);
    const cplx xq = x[j], xu = x[n + j];
    fma_acc(y1, e[0], xq);
    fma_acc(y1, e[1], xu);
    fma_acc(y2, e[2], xq);
    fma_acc(y2, e[3], xu);
  }
  y[i] = y1;
  y[n + i] = y2;
}

void launch_kblock(hipStream_t st, int eq, const PointsDev& P, const MediumDev* media, const KJob* jobs,
                   const KTile* tiles, int ntiles, const int* rpt, const int* rmap1, const int* rmap2,
                   const int* cpt, const int* cmap1, const int* cmap2) {
  if (ntiles <= 0) return;
  if (eq == kEqPmchwt)
    hipLaunchKernelGGL(k_kblock<kEqPmchwt>, dim3(ntiles), dim3(256), 0, st, P, media, jobs, tiles, rpt, rmap1,
                       rmap2, cpt, cmap1, cmap2);
  else if (eq == kEqBurtonMiller)
    hipLaunchKernelGGL(k_kblock<kEqBurtonMiller>, dim3(ntiles), dim3(256), 0, st, P, media, jobs, tiles, rpt,
                       rmap1, rmap2, cpt, cmap1, cmap2);
  else
    hipLaunchKernelGGL(k_kblock<kEqMuller>, dim3(ntiles), dim3(256), 0, st, P, media, jobs, tiles, rpt, rmap1,
                       rmap2, cpt, cmap1, cmap2);
  HIPCHK(hipGetLastError());
}

void launch_geometry(hipStream_t st, int n, const double* x, const double* dx, const double* ddx, double* px,
                     double* py, double* nx, double* ny, double* w, double* kappa) {
  hipLaunchKernelGGL(k_geometry, dim3(cdiv_int(n, 256)), dim3(256), 0, st, n, x, dx, ddx, px, py, nx, ny, w,
                     kappa);
  HIPCHK(hipGetLastError());
}

void launch_rhs_plane(hipStream_t st, int n, const PointsDev& P, const MediumDev& md, double angle, cplx* b) {
  hipLaunchKernelGGL(k_rhs_plane, dim3(cdiv_int(n, 256)), dim3(256), 0, st, n, P, md, cos(angle), sin(angle), b);
  HIPCHK(hipGetLastError());
}

void launch_plane_incident(hipStream_t st, int n, const PointsDev& P, const MediumDev& md, double angle, cplx* uin,
                           cplx* qin) {
  hipLaunchKernelGGL(k_plane_incident, dim3(cdiv_int(n, 256)), dim3(256), 0, st, n, P, md, cos(angle), sin(angle),
                     uin, qin);
  HIPCHK(hipGetLastError());
}

void launch_rhs_incident(hipStream_t st, int n, const PointsDev& P, const MediumDev& md, const cplx* uin,
                         const cplx* qin, int ldi, cplx* b, int ldb, int nrhs) {
  hipLaunchKernelGGL(k_rhs_incident, dim3(cdiv_int(n, 256), nrhs), dim3(256), 0, st, n, P, md, uin, qin, ldi, b,
                     ldb);
  HIPCHK(hipGetLastError());
}

void launch_split_traces(hipStream_t st, int n, const cplx* x, int ldx, cplx* q, cplx* u, int ldo, int nrhs) {
  hipLaunchKernelGGL(k_split_traces, dim3(cdiv_int(n, 256), nrhs), dim3(256), 0, st, n, x, ldx, q, u, ldo);
  HIPCHK(hipGetLastError());
}

void launch_bessel(hipStream_t st, int n, const double* z, double* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_bessel, dim3(cdiv_int(n, 256)), dim3(256), 0, st, n, z, out);
  HIPCHK(hipGetLastError());
}

void launch_matvec_direct(hipStream_t st, const PointsDev& P, const MediumDev& md, const cplx* x, cplx* y) {
  const dim3 g(cdiv_int(P.n_boundary, 256));
  if (md.eq == kEqPmchwt)
    hipLaunchKernelGGL(k_matvec_direct<kEqPmchwt>, g, dim3(256), 0, st, P, md, x, y);
  else if (md.eq == kEqBurtonMiller)
    hipLaunchKernelGGL(k_matvec_direct<kEqBurtonMiller>, g, dim3(256), 0, st, P, md, x, y);
  else
    hipLaunchKernelGGL(k_matvec_direct<kEqMuller>, g, dim3(256), 0, st, P, md, x, y);
  HIPCHK(hipGetLastError());
}

}  // namespace symhss

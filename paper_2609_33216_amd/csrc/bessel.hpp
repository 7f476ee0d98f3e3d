// Bessel functions J0, Y0, J1, Y1 of real positive argument in FP64, for the
// Hankel functions H_n^(1) = J_n + i Y_n of the 2-D Helmholtz fundamental
// solution G_k = (i/4) H0^(1)(k r) (paper Section 3.1).
//
// One call returns all four values and the regular part of Y1,
//   y1r(z) = Y1(z) + 2/(pi z),
// so that differences k0 Y1(k0 r) - k1 Y1(k1 r), whose 2/(pi r) poles cancel
// exactly, are formed without cancellation.
//
// Three regimes, each from published mathematics:
//   z <= Z_SERIES : ascending series (DLMF 10.2.2 for J; DLMF 10.8.1 and
//                   10.8.2 for Y, with psi(m+1) = -gamma + H_m).
//   Z_SERIES < z < Z_ASYMP : Miller's backward recurrence for J_n
//                   (DLMF 3.6(vi)), normalised by J0 + 2 sum J_2k = 1
//                   (DLMF 10.12.4), with Neumann's series
//                   Y0 = (2/pi)(ln(z/2)+gamma) J0 - (4/pi) sum (-1)^k J_2k / k
//                   (DLMF 10.23.9) and its derivative for Y1 = -Y0'.
//   z >= Z_ASYMP  : Hankel's asymptotic expansion (DLMF 10.17.3, 10.17.4)
//                   in the P/Q form, Horner-evaluated in 1/z^2.
// Series and expansion coefficients are generated at compile time from their
// closed forms (constexpr), so the device code holds no literal tables.
#pragma once

#include <cmath>

#ifndef SYMHSS_HD
#define SYMHSS_HD __host__ __device__
#endif

namespace symhss {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoOverPi = 0.63661977236758134308;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kSqrtHalf = 0.70710678118654752440;
constexpr double kZSeries = 4.0;
constexpr double kZAsymp = 25.0;

struct JY01 {
  double j0, y0, j1, y1, y1r;  // y1r = Y1 + 2/(pi z)
};

// Coefficients of the ascending series as polynomials in t = -z^2/4, built at
// compile time from their definitions:
//   a0_m = 1/(m!)^2,  a1_m = 1/(m!(m+1)!),  b0_m = H_m/(m!)^2,
//   b1_m = (H_m + H_{m+1})/(m!(m+1)!),  H_m = 1 + 1/2 + ... + 1/m.
constexpr int kSeriesTerms = 19;  // m = 0..18: last term < 1e-17 of the sum for z <= 4
struct SeriesCoef {
  double a0[kSeriesTerms], a1[kSeriesTerms], b0[kSeriesTerms], b1[kSeriesTerms];
};
constexpr SeriesCoef make_series_coef() {
  SeriesCoef c{};
  double f = 1.0, h = 0.0;
  for (int m = 0; m < kSeriesTerms; ++m) {
    if (m > 0) {
      f *= m;
      h += 1.0 / m;
    }
    const double f1 = f * (m + 1);
    const double h1 = h + 1.0 / (m + 1);
    c.a0[m] = 1.0 / (f * f);
    c.a1[m] = 1.0 / (f * f1);
    c.b0[m] = h / (f * f);
    c.b1[m] = (h + h1) / (f * f1);
  }
  return c;
}
constexpr SeriesCoef kSeries = make_series_coef();

// Ascending series, Horner form.  With t = -z^2/4:
//   J0  = sum a0_m t^m
//   J1  = (z/2) sum a1_m t^m
//   Y0  = (2/pi)[(ln(z/2)+gamma) J0 - sum b0_m t^m]
//   Y1r = (2/pi)(ln(z/2)+gamma) J1 - (z/(2pi)) sum b1_m t^m
SYMHSS_HD inline JY01 jy01_series(double z) {
  const double t = -0.25 * z * z;
  double pj0 = kSeries.a0[kSeriesTerms - 1], pj1 = kSeries.a1[kSeriesTerms - 1];
  double py0 = kSeries.b0[kSeriesTerms - 1], py1 = kSeries.b1[kSeriesTerms - 1];
  // coefficients come from scalar loads of the constant table: fully unrolled,
  // the 76 FP64 literals would exhaust the scalar register file
#pragma unroll 2
  for (int m = kSeriesTerms - 2; m >= 0; --m) {
    pj0 = fma(pj0, t, kSeries.a0[m]);
    pj1 = fma(pj1, t, kSeries.a1[m]);
    py0 = fma(py0, t, kSeries.b0[m]);
    py1 = fma(py1, t, kSeries.b1[m]);
  }
  JY01 r;
  const double lg = std::log(0.5 * z) + kEulerGamma;
  r.j0 = pj0;
  r.j1 = 0.5 * z * pj1;
  r.y0 = kTwoOverPi * (lg * r.j0 - py0);
  r.y1r = kTwoOverPi * lg * r.j1 - z * (0.5 / kPi) * py1;
  r.y1 = r.y1r - kTwoOverPi / z;
  return r;
}

// Miller backward recurrence j_{n-1} = (2n/z) j_n - j_{n+1} from an even start
// order M with j_{M+1} = 0, two orders per iteration (n = 2k even, then
// 2k - 1), accumulating the normalisation sum and the Neumann sums:
//   S0 = sum_{k>=1} (-1)^k j_2k / k
//   S1 = sum_{k>=1} (-1)^k (j_{2k-1} - j_{2k+1}) / k
// Y1 = -Y0' = -(2/pi) J0/z + (2/pi)(ln(z/2)+gamma) J1 + (2/pi) S1/norm.
SYMHSS_HD inline JY01 jy01_miller(double z) {
  const int K = (int)(0.5 * (z + 6.0 * std::cbrt(z) + 18.0));  // M = 2K
  const double twoz = 2.0 / z;
  double jp1 = 0.0, jn = 1e-30;  // j_{2K+1}, j_{2K}
  double norm = 0.0, s0 = 0.0, s1 = 0.0;
  double sg = (K & 1) ? -1.0 : 1.0;  // (-1)^k
  for (int k = K; k >= 1; --k) {
    const double ik = 1.0 / k;
    const int n = 2 * k;
    // even order n = 2k: jn = j_2k, jp1 = j_{2k+1}
    norm += 2.0 * jn;
    s0 += sg * jn * ik;
    const double jm1 = n * twoz * jn - jp1;  // j_{2k-1}
    s1 += sg * (jm1 - jp1) * ik;
    const double jm2 = (n - 1) * twoz * jm1 - jn;  // j_{2k-2}
    jp1 = jm1;
    jn = jm2;
    sg = -sg;
  }
  norm += jn;  // + j_0
  const double inv = 1.0 / norm;
  JY01 r;
  r.j0 = jn * inv;
  r.j1 = jp1 * inv;
  const double lg = std::log(0.5 * z) + kEulerGamma;
  r.y0 = kTwoOverPi * (lg * r.j0 - 2.0 * s0 * inv);
  r.y1 = kTwoOverPi * (-r.j0 / z + lg * r.j1 + s1 * inv);
  r.y1r = r.y1 + kTwoOverPi / z;
  return r;
}

// Hankel's expansion (DLMF 10.17.1-4): for nu = 0, 1,
//   a_k(nu) = prod_{j=1..k} (4 nu^2 - (2j-1)^2) / (k! 8^k),
//   P = sum_k (-1)^k a_2k / z^2k,  Q = sum_k (-1)^k a_{2k+1} / z^{2k+1},
//   J = sqrt(2/(pi z)) (P cos w - Q sin w),  Y = sqrt(2/(pi z)) (P sin w + Q cos w),
//   w = z - nu pi/2 - pi/4.
// P and Q are evaluated as polynomials in u = 1/z^2 (Horner) with the
// coefficients (-1)^k a_2k and (-1)^k a_{2k+1} built at compile time; 13 terms
// each (a_0 .. a_25) reach 1e-16 for z >= 25.
constexpr int kAsympTerms = 13;
struct AsympCoef {
  double p0[kAsympTerms], q0[kAsympTerms], p1[kAsympTerms], q1[kAsympTerms];
};
constexpr AsympCoef make_asymp_coef() {
  AsympCoef c{};
  double a0 = 1.0, a1 = 1.0;  // a_k(0), a_k(1)
  for (int k = 0; k < 2 * kAsympTerms; ++k) {
    if (k > 0) {
      const double o = (double)(2 * k - 1) * (double)(2 * k - 1);
      a0 *= (0.0 - o) / (8.0 * k);
      a1 *= (4.0 - o) / (8.0 * k);
    }
    const int h = k / 2;
    const double sg = (h & 1) ? -1.0 : 1.0;
    if ((k & 1) == 0) {
      c.p0[h] = sg * a0;
      c.p1[h] = sg * a1;
    } else {
      c.q0[h] = sg * a0;
      c.q1[h] = sg * a1;
    }
  }
  return c;
}
constexpr AsympCoef kAsymp = make_asymp_coef();

SYMHSS_HD inline JY01 jy01_asymp(double z) {
  const double iz = 1.0 / z;
  const double u = iz * iz;
  double p0 = kAsymp.p0[kAsympTerms - 1], q0 = kAsymp.q0[kAsympTerms - 1];
  double p1 = kAsymp.p1[kAsympTerms - 1], q1 = kAsymp.q1[kAsympTerms - 1];
#pragma unroll 2
  for (int k = kAsympTerms - 2; k >= 0; --k) {
    p0 = fma(p0, u, kAsymp.p0[k]);
    q0 = fma(q0, u, kAsymp.q0[k]);
    p1 = fma(p1, u, kAsymp.p1[k]);
    q1 = fma(q1, u, kAsymp.q1[k]);
  }
  q0 *= iz;
  q1 *= iz;
  double s, c;
#if defined(__HIP_DEVICE_COMPILE__)
  sincos(z, &s, &c);
#else
  s = std::sin(z);
  c = std::cos(z);
#endif
  const double cw0 = (c + s) * kSqrtHalf;  // cos(z - pi/4)
  const double sw0 = (s - c) * kSqrtHalf;  // sin(z - pi/4)
  const double cw1 = sw0;                  // cos(z - 3pi/4)
  const double sw1 = -cw0;                 // sin(z - 3pi/4)
  const double amp = std::sqrt(kTwoOverPi * iz);
  JY01 r;
  r.j0 = amp * (p0 * cw0 - q0 * sw0);
  r.y0 = amp * (p0 * sw0 + q0 * cw0);
  r.j1 = amp * (p1 * cw1 - q1 * sw1);
  r.y1 = amp * (p1 * sw1 + q1 * cw1);
  r.y1r = r.y1 + kTwoOverPi * iz;
  return r;
}

SYMHSS_HD inline JY01 jy01(double z) {
  if (z <= kZSeries) return jy01_series(z);
  if (z < kZAsymp) return jy01_miller(z);
  return jy01_asymp(z);
}

}  // namespace symhss

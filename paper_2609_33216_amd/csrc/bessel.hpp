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
//                   in the P/Q (modulus-phase) form.
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

// Ascending series.  With t = -z^2/4:
//   J0  = sum t^m / (m!)^2
//   J1  = (z/2) sum t^m / (m! (m+1)!)
//   Y0  = (2/pi)(ln(z/2)+gamma) J0 - (2/pi) sum_{m>=1} H_m t^m / (m!)^2
//   Y1r = (2/pi)(ln(z/2)+gamma) J1 - (z/(2pi)) sum (H_m + H_{m+1}) t^m / (m!(m+1)!)
SYMHSS_HD inline JY01 jy01_series(double z) {
  const double t = -0.25 * z * z;
  double a = 1.0;   // t^m/(m!)^2
  double b = 1.0;   // t^m/(m!(m+1)!)
  double hm = 0.0;  // H_m
  double sj0 = 1.0, sj1 = 1.0, sy0 = 0.0, sy1 = 1.0;  // m = 0 terms (H_0 + H_1 = 1)
#pragma unroll
  for (int m = 1; m <= 18; ++m) {
    const double inv = 1.0 / m;
    a *= t * inv * inv;
    b *= t * inv / (m + 1);
    hm += inv;
    const double hm1 = hm + 1.0 / (m + 1);
    sj0 += a;
    sj1 += b;
    sy0 += hm * a;
    sy1 += (hm + hm1) * b;
  }
  JY01 r;
  const double lg = std::log(0.5 * z) + kEulerGamma;
  r.j0 = sj0;
  r.j1 = 0.5 * z * sj1;
  r.y0 = kTwoOverPi * (lg * r.j0 - sy0);
  r.y1r = kTwoOverPi * lg * r.j1 - z * (0.5 / kPi) * sy1;
  r.y1 = r.y1r - kTwoOverPi / z;
  return r;
}

// Miller backward recurrence j_{n-1} = (2n/z) j_n - j_{n+1} from an even start
// order M with j_{M+1} = 0, accumulating the normalisation sum and the two
// Neumann sums on the way down:
//   S0 = sum_{k>=1} (-1)^k j_2k / k
//   S1 = sum_{k>=1} (-1)^k (j_{2k-1} - j_{2k+1}) / k
// Y1 = -Y0' = -(2/pi) J0/z + (2/pi)(ln(z/2)+gamma) J1 + (2/pi) S1/norm.
SYMHSS_HD inline JY01 jy01_miller(double z) {
  const int M = 2 * (int)(0.5 * (z + 6.0 * std::cbrt(z) + 18.0));
  const double twoz = 2.0 / z;
  double jp2 = 0.0, jp1 = 0.0, jn = 1e-30;  // j_{n+2}, j_{n+1}, j_n at n = M
  double norm = 0.0, s0 = 0.0, s1 = 0.0;
  for (int n = M; n >= 1; --n) {
    if ((n & 1) == 0) {
      const int k = n >> 1;
      const double t = jn / k;
      norm += 2.0 * jn;
      s0 += (k & 1) ? -t : t;
    } else {
      const int k = (n + 1) >> 1;  // n = 2k - 1
      const double t = (jn - jp2) / k;
      s1 += (k & 1) ? -t : t;
    }
    const double jm1 = n * twoz * jn - jp1;
    jp2 = jp1;
    jp1 = jn;
    jn = jm1;
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

// Hankel's expansion: for nu = 0, 1 with mu = 4 nu^2,
//   P = sum_k (-1)^k a_2k / z^2k,  Q = sum_k (-1)^k a_{2k+1} / z^{2k+1},
//   a_k / z^k = a_{k-1} / z^{k-1} * (mu - (2k-1)^2) / (8 k z),
//   J = sqrt(2/(pi z)) (P cos w - Q sin w),  Y = sqrt(2/(pi z)) (P sin w + Q cos w),
//   w = z - nu pi/2 - pi/4.
SYMHSS_HD inline JY01 jy01_asymp(double z) {
  const double inv8z = 0.125 / z;
  double p0 = 1.0, q0 = 0.0, p1 = 1.0, q1 = 0.0;
  double t0 = 1.0, t1 = 1.0;
#pragma unroll
  for (int k = 1; k <= 26; ++k) {
    const double o = (double)(2 * k - 1) * (double)(2 * k - 1);
    t0 *= (0.0 - o) * inv8z / k;
    t1 *= (4.0 - o) * inv8z / k;
    // sign pattern of i^k: k = 1 -> +Q, 2 -> -P, 3 -> -Q, 4 -> +P ...
    const int km = k & 3;
    if (km == 1) { q0 += t0; q1 += t1; }
    else if (km == 2) { p0 -= t0; p1 -= t1; }
    else if (km == 3) { q0 -= t0; q1 -= t1; }
    else { p0 += t0; p1 += t1; }
  }
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
  const double amp = std::sqrt(kTwoOverPi / z);
  JY01 r;
  r.j0 = amp * (p0 * cw0 - q0 * sw0);
  r.y0 = amp * (p0 * sw0 + q0 * cw0);
  r.j1 = amp * (p1 * cw1 - q1 * sw1);
  r.y1 = amp * (p1 * sw1 + q1 * cw1);
  r.y1r = r.y1 + kTwoOverPi / z;
  return r;
}

SYMHSS_HD inline JY01 jy01(double z) {
  if (z <= kZSeries) return jy01_series(z);
  if (z < kZAsymp) return jy01_miller(z);
  return jy01_asymp(z);
}

}  // namespace symhss

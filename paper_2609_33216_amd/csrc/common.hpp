// Shared types of the HIP path: complex FP64 arithmetic, device descriptors
// and launch helpers.  Host and device code both include this header.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <type_traits>

namespace symhss {

struct cplx {
  double re, im;
};

__host__ __device__ inline cplx mk(double r, double i) { return cplx{r, i}; }
__host__ __device__ inline cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplx operator-(cplx a) { return {-a.re, -a.im}; }
__host__ __device__ inline cplx operator*(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
__host__ __device__ inline cplx conj(cplx a) { return {a.re, -a.im}; }
__host__ __device__ inline double abs2(cplx a) { return a.re * a.re + a.im * a.im; }
// a += b * c
__host__ __device__ inline void fma_acc(cplx& a, cplx b, cplx c) {
  a.re = fma(b.re, c.re, fma(-b.im, c.im, a.re));
  a.im = fma(b.re, c.im, fma(b.im, c.re, a.im));
}
// a += conj(b) * c
__host__ __device__ inline void fma_conj_acc(cplx& a, cplx b, cplx c) {
  a.re = fma(b.re, c.re, fma(b.im, c.im, a.re));
  a.im = fma(b.re, c.im, fma(-b.im, c.re, a.im));
}
__host__ __device__ inline cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.im + b.re * r;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

// 1 / z as conj(z) / |z|^2: one real division (pivots of the LU panels,
// whose magnitudes are far from the overflow range of |z|^2).
__host__ __device__ inline cplx crecip(cplx z) {
  const double d = 1.0 / (z.re * z.re + z.im * z.im);
  return {z.re * d, -z.im * d};
}

// Complex FP32 (mixed-precision factorisation) with the same operations.
struct cplxf {
  float re, im;
};
__host__ __device__ inline cplxf operator+(cplxf a, cplxf b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplxf operator-(cplxf a, cplxf b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplxf operator-(cplxf a) { return {-a.re, -a.im}; }
__host__ __device__ inline cplxf operator*(cplxf a, cplxf b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cplxf operator*(double s, cplxf a) { return {(float)s * a.re, (float)s * a.im}; }
__host__ __device__ inline cplxf conj(cplxf a) { return {a.re, -a.im}; }
__host__ __device__ inline float abs2(cplxf a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ inline void fma_acc(cplxf& a, cplxf b, cplxf c) {
  a.re = fmaf(b.re, c.re, fmaf(-b.im, c.im, a.re));
  a.im = fmaf(b.re, c.im, fmaf(b.im, c.re, a.im));
}
__host__ __device__ inline void fma_conj_acc(cplxf& a, cplxf b, cplxf c) {
  a.re = fmaf(b.re, c.re, fmaf(b.im, c.im, a.re));
  a.im = fmaf(b.re, c.im, fmaf(-b.im, c.re, a.im));
}
// Accesses through pointers known to address global memory.  A pointer read
// from a descriptor in memory is generic, so the compiler emits flat
// instructions for it; a flat access counts against the LDS counter too, and
// the compiler then waits for every flat access in flight before it uses an
// LDS result (and the reverse), so that global loads cannot overlap LDS work
// or each other.  These helpers load and store through the global address
// space instead.  Only for pointers into device memory (never LDS or stack).
#define SYMHSS_GLOBAL_AS __attribute__((address_space(1)))
typedef double symhss_v2d __attribute__((ext_vector_type(2)));
typedef float symhss_v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cplx ldg(const cplx* p) {
  const symhss_v2d v = *(const SYMHSS_GLOBAL_AS symhss_v2d*)p;
  return cplx{v.x, v.y};
}
__device__ __forceinline__ void stg(cplx* p, cplx c) {
  const symhss_v2d v = {c.re, c.im};
  *(SYMHSS_GLOBAL_AS symhss_v2d*)p = v;
}
__device__ __forceinline__ cplxf ldg(const cplxf* p) {
  const symhss_v2f v = *(const SYMHSS_GLOBAL_AS symhss_v2f*)p;
  return cplxf{v.x, v.y};
}
__device__ __forceinline__ void stg(cplxf* p, cplxf c) {
  const symhss_v2f v = {c.re, c.im};
  *(SYMHSS_GLOBAL_AS symhss_v2f*)p = v;
}
__device__ __forceinline__ int ldg(const int* p) { return *(const SYMHSS_GLOBAL_AS int*)p; }
__device__ __forceinline__ void stg(int* p, int v) { *(SYMHSS_GLOBAL_AS int*)p = v; }
__device__ __forceinline__ double ldg(const double* p) { return *(const SYMHSS_GLOBAL_AS double*)p; }
__device__ __forceinline__ void stg(double* p, double v) { *(SYMHSS_GLOBAL_AS double*)p = v; }

__host__ __device__ inline cplxf cdiv(cplxf a, cplxf b) {
  if (fabsf(b.re) >= fabsf(b.im)) {
    const float r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const float r = b.re / b.im, d = b.im + b.re * r;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

__host__ __device__ inline cplxf crecip(cplxf z) {
  const float d = 1.0f / (z.re * z.re + z.im * z.im);
  return {z.re * d, -z.im * d};
}

// Boundary and proxy points, structure of arrays.  Index < n_boundary is a
// boundary node (the nodes of all boundaries of a batch, one after another);
// larger indices are proxy points of the current level.
struct PointsDev {
  const double* x;
  const double* y;
  const double* nx;
  const double* ny;
  const double* w;
  const double* kappa;  // curvature (boundary nodes only)
  int n_boundary;
};

// Medium constants.  eps0, eps1 and the wavenumbers; the remaining fields are
// the point-independent parts of the one-point corrected diagonals.
struct MediumDev {
  double k0, k1, eps0, eps1;
  double g0c, g1c;      // ln(k/2) + gamma for k0, k1
  double nd_re, nd_im;  // N_k0 - N_k1 diagonal without the -(Delta/4pi) ln(w/2pi) term
  double delta;         // k0^2 - k1^2
  int row_scaled;       // 1: rows scaled by w (eq. symmetric_muller / symmetric_pmchwt); 0: unscaled
  int eq;               // kEqMuller, kEqPmchwt or kEqBurtonMiller
  double ie0, ie1;      // 1 / eps0, 1 / eps1 (PMCHWT)
  // individual (hypersingular) N_k diagonal without the point-dependent
  // -pi/(6 w^2) + kappa^2/(24 pi) - (k^2/4pi) ln(w/2pi):
  // i k^2/8 - (k^2/4pi)(ln(k/2) + gamma - 1/2)
  double n0_re, n0_im, n1_re, n1_im;
  double al_re, al_im;  // Burton-Miller coupling alpha = i / k0
};

// Which boundary integral system the entries belong to.
constexpr int kEqMuller = 0;        // eq. symmetric_muller / naive_muller
constexpr int kEqPmchwt = 1;        // eq. symmetric_pmchwt / naive_pmchwt
constexpr int kEqBurtonMiller = 2;  // eq. bm, columns in [q; u] order

// One block job of the kernel-block generator: the 2x2 Muller-like block
// between row points and column points, written into a column-major matrix.
// For row point a: rmap1[a] / rmap2[a] is the output row of its first /
// second equation (-1: not wanted).  For column point b: cmap1[b] / cmap2[b]
// is the output column of its q / u unknown.  mode 0 writes out[rmap, cmap];
// mode 1 also writes the transposed position out[cmap, rmap] (valid when row
// and column positions share one index space and the matrix is symmetric);
// mode 2 writes only out[cmap, rmap] (a block stored transposed, e.g. M_L^T).
struct KJob {
  cplx* out;
  int ld;
  int nr, nc;
  int roff, coff;  // offsets into the row / column index arrays
  int mode;
  int med;         // index of the medium (one per boundary of a batch)
};

struct KTile {
  int job, r0, c0, pad;
};

// Arg-max over the 64 lanes of a wavefront: the largest v (NaN never wins),
// the lowest i among equal v; every lane receives the result.  Within each
// 16-lane row the pairs are exchanged by DPP lane permutations (quad
// exchanges by 1 and 2, then the half-row and row mirrors: after each step
// every lane holds the result over the lanes combined so far); the four row
// results are then read with readlane and combined in the same order on
// every lane.
template <int CTRL>
__device__ __forceinline__ void argmax_dpp_step(double& v, int& i) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  const int oi = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xF, 0xF, false);
  const double ov = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  argmax_dpp_step<0xB1>(v, i);   // quad_perm [1, 0, 3, 2]
  argmax_dpp_step<0x4E>(v, i);   // quad_perm [2, 3, 0, 1]
  argmax_dpp_step<0x141>(v, i);  // row_half_mirror
  argmax_dpp_step<0x140>(v, i);  // row_mirror
  const long long b = __double_as_longlong(v);
  double bv = 0.0;
  int bi = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int lo = __builtin_amdgcn_readlane((int)b, 16 * r);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * r);
    const int ri = __builtin_amdgcn_readlane(i, 16 * r);
    const double rv = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    if (r == 0 || rv > bv || (rv == bv && ri < bi)) {
      bv = rv;
      bi = ri;
    }
  }
  v = bv;
  i = bi;
}

// Arg-max by 32-bit keys: a candidate's key is the upper word of its
// non-negative FP64 magnitude (monotone in the magnitude, NaN above +inf)
// with the low IDX_BITS + 1 bits replaced by a marker bit and
// 2^IDX_BITS - 1 - i, so that the largest key names the largest magnitude
// and, among magnitudes equal to about 2^-(19 - IDX_BITS) relative, the lowest
// index i (0 <= i < 2^IDX_BITS).  Key 0 means "no candidate".  One 32-bit
// maximum per exchange instead of a value and an index.
template <int IDX_BITS>
__device__ __forceinline__ unsigned argmax_key(double v, int i) {
  if (!(v >= 0.0) && v == v) return 0u;  // negative: no candidate (NaN is a candidate)
  constexpr unsigned low = (2u << IDX_BITS) - 1u;
  const unsigned hi = (unsigned)(__double_as_longlong(v) >> 32);
  return (hi & ~low) | (1u << IDX_BITS) | ((1u << IDX_BITS) - 1u - (unsigned)i);
}
template <int IDX_BITS>
__device__ __forceinline__ int argmax_key_index(unsigned k) {
  return (int)((1u << IDX_BITS) - 1u - (k & ((1u << IDX_BITS) - 1u)));
}
template <int CTRL>
__device__ __forceinline__ unsigned dpp_max_u32(unsigned k) {
  const unsigned o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, CTRL, 0xF, 0xF, false);
  return o > k ? o : k;
}
// Largest key over the 64 lanes (every lane receives it): DPP exchanges
// within rows of 16, then the four rows by readlane.
__device__ __forceinline__ unsigned wave_max_key(unsigned k) {
  k = dpp_max_u32<0xB1>(k);   // quad_perm [1, 0, 3, 2]
  k = dpp_max_u32<0x4E>(k);   // quad_perm [2, 3, 0, 1]
  k = dpp_max_u32<0x141>(k);  // row_half_mirror
  k = dpp_max_u32<0x140>(k);  // row_mirror
  const unsigned a = __builtin_amdgcn_readlane(k, 0), b = __builtin_amdgcn_readlane(k, 16);
  const unsigned c = __builtin_amdgcn_readlane(k, 32), d = __builtin_amdgcn_readlane(k, 48);
  const unsigned ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// Sum over the 64 lanes of a wavefront; every lane receives the same value.
// Row sums by the DPP exchanges of wave_argmax, then the four row sums in
// lane order.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ float readlane_real(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double readlane_real(double v, int lane) { return readlane_f64(v, lane); }

__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return ((readlane_f64(v, 0) + readlane_f64(v, 16)) + readlane_f64(v, 32)) + readlane_f64(v, 48);
}

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
  }
}

#define HIPCHK(x) ::symhss::hip_check((x), #x)

inline int cdiv_int(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace symhss

// Device math for the per-point path: sine/cosine of reduced arguments,
// rotation by small angles, and fast reciprocals.
//
// sincos_rr: any |x| whose multiple k of pi/2 is below 2^53 (the error of the
// reduction grows like k * 2e-33; for the angles of this model, below 1e5 rad
// in practice, it is negligible).  x = k*pi/2 + r with k = rint(2x/pi) and r by
// a two-constant Cody-Waite step (the product k*pi/2_hi is exact inside the
// fused multiply-add), |r| <= pi/4, then the Taylor series of sin and cos
// (1/n! coefficients): through r^15 / r^16 in double (truncation below
// 5e-17 absolute), r^9 / r^10 in float (below 2e-9).  The quadrant k mod 4
// permutes and signs the pair.
//
// sincos_mx: argument in double, reduction in double, series in float: the
// reduced angle has no float rounding beyond its final conversion.
//
// rotate_small: (sin x, cos x) -> (sin(x+d), cos(x+d)) by angle addition with
// the series of sin d and cos d; used for |d| <= kRotMax, exact to rounding
// there (double: d^9/9! < 6e-18 at |d| = 0.05).
#pragma once

#include <hip/hip_runtime.h>

namespace sgp4mi {

constexpr double kTwoOverPi = 0.63661977236758134308;
constexpr double kPio2Hi = 1.5707963267948966192;    // double nearest pi/2
constexpr double kPio2Lo = 6.123233995736766036e-17;  // pi/2 - kPio2Hi
constexpr double kRotMax = 0.05;

template <class T>
__device__ __forceinline__ void quadrant(int q, T sr, T cr, T* s, T* c) {
  T ss = (q & 1) ? cr : sr;
  T cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// Double-precision coefficients live in constant memory: gfx9 VALU
// instructions take no 64-bit literals, and scalar-register operands (one per
// instruction) avoid holding every coefficient in a vector register pair.
__constant__ double kSinCos64[17] = {
    -7.6471637318198164759e-13,  // -1/15!
    1.6059043836821614599e-10,   // 1/13!
    -2.5052108385441718775e-8,   // -1/11!
    2.7557319223985890653e-6,    // 1/9!
    -1.9841269841269841270e-4,   // -1/7!
    8.3333333333333333333e-3,    // 1/5!
    -1.6666666666666666667e-1,   // -1/3!
    4.7794773323873852974e-14,   // 1/16!
    -1.1470745597729724714e-11,  // -1/14!
    2.0876756987868098979e-9,    // 1/12!
    -2.7557319223985890653e-7,   // -1/10!
    2.4801587301587301587e-5,    // 1/8!
    -1.3888888888888888889e-3,   // -1/6!
    4.1666666666666666667e-2,    // 1/4!
    0.63661977236758134308,      // 2/pi
    1.5707963267948966192,       // pi/2 (double nearest)
    6.123233995736766036e-17,    // pi/2 minus the above
};

__device__ __forceinline__ void series(double r, double* s, double* c) {
  const double* k = kSinCos64;
  const double r2 = r * r;
  double ps = fma(k[0], r2, k[1]);
  ps = fma(ps, r2, k[2]);
  ps = fma(ps, r2, k[3]);
  ps = fma(ps, r2, k[4]);
  ps = fma(ps, r2, k[5]);
  ps = fma(ps, r2, k[6]);
  *s = fma(ps * r2, r, r);
  double pc = fma(k[7], r2, k[8]);
  pc = fma(pc, r2, k[9]);
  pc = fma(pc, r2, k[10]);
  pc = fma(pc, r2, k[11]);
  pc = fma(pc, r2, k[12]);
  pc = fma(pc, r2, k[13]);
  pc = fma(pc, r2, -0.5);
  *c = fma(pc, r2, 1.0);
}

__device__ __forceinline__ void series(float r, float* s, float* c) {
  const float r2 = r * r;
  float ps = 2.7557319224e-6f;                  // 1/9!
  ps = fmaf(ps, r2, -1.9841269841e-4f);         // -1/7!
  ps = fmaf(ps, r2, 8.3333333333e-3f);          // 1/5!
  ps = fmaf(ps, r2, -1.6666666667e-1f);         // -1/3!
  *s = fmaf(ps * r2, r, r);
  float pc = -2.7557319224e-7f;                 // -1/10!
  pc = fmaf(pc, r2, 2.4801587302e-5f);          // 1/8!
  pc = fmaf(pc, r2, -1.3888888889e-3f);         // -1/6!
  pc = fmaf(pc, r2, 4.1666666667e-2f);          // 1/4!
  pc = fmaf(pc, r2, -0.5f);
  *c = fmaf(pc, r2, 1.0f);
}

// k mod 4 taken in floating point (exact for any integral k below 2^53, or
// 2^24 in float), so the quadrant stays right when k exceeds the int range.
__device__ __forceinline__ int quad_of(double k) { return int(fma(-4.0, floor(k * 0.25), k)); }
__device__ __forceinline__ int quad_of(float k) { return int(fmaf(-4.0f, floorf(k * 0.25f), k)); }

__device__ __forceinline__ void sincos_rr(double x, double* s, double* c) {
  const double k = rint(x * kSinCos64[14]);
  double r = fma(-k, kSinCos64[15], x);
  r = fma(-k, kSinCos64[16], r);
  double sr, cr;
  series(r, &sr, &cr);
  quadrant(quad_of(k), sr, cr, s, c);
}

__device__ __forceinline__ void sincos_rr(float x, float* s, float* c) {
  const float k = rintf(x * 0.63661977236758134308f);
  float r = fmaf(-k, 1.57079637050628662109375f, x);   // float nearest pi/2
  r = fmaf(-k, -4.37113900018624283e-8f, r);            // pi/2 minus that
  float sr, cr;
  series(r, &sr, &cr);
  quadrant(quad_of(k), sr, cr, s, c);
}

__device__ __forceinline__ void sincos_mx(double x, float* s, float* c) {
  const double k = rint(x * kSinCos64[14]);
  double r = fma(-k, kSinCos64[15], x);
  r = fma(-k, kSinCos64[16], r);
  float sr, cr;
  series(float(r), &sr, &cr);
  quadrant(quad_of(k), sr, cr, s, c);
}

__device__ __forceinline__ void small_sc(double d, double* sd, double* cd) {
  const double* k = kSinCos64;
  const double d2 = d * d;
  double ps = fma(d2, k[4], k[5]);
  ps = fma(ps, d2, k[6]);
  *sd = fma(ps * d2, d, d);
  double pc = fma(d2, k[11], k[12]);
  pc = fma(pc, d2, k[13]);
  pc = fma(pc, d2, -0.5);
  *cd = fma(pc, d2, 1.0);
}

__device__ __forceinline__ void small_sc(float d, float* sd, float* cd) {
  const float d2 = d * d;
  float ps = fmaf(d2, 8.3333333333e-3f, -1.6666666667e-1f);
  *sd = fmaf(ps * d2, d, d);
  float pc = fmaf(d2, 4.1666666667e-2f, -0.5f);
  *cd = fmaf(pc, d2, 1.0f);
}

template <class T>
__device__ __forceinline__ void rotate_small(T* s, T* c, T d) {
  T sd, cd;
  small_sc(d, &sd, &cd);
  const T s0 = *s, c0 = *c;
  *s = s0 * cd + c0 * sd;
  *c = c0 * cd - s0 * sd;
}

// Reciprocal: hardware estimate refined by two Newton steps (double) or the
// hardware estimate alone (float, about 1 ulp).
__device__ __forceinline__ double rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

}  // namespace sgp4mi

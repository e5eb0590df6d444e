// Device math for the per-point path: sine/cosine of any angle of the
// model, rotation by small angles, and fast reciprocals.
//
// sincos_rr: y = x - 2*pi*k with k = rint(x / 2*pi) (a two-part 2*pi, the
// product exact inside the fused multiply-add), then, in float, the Taylor
// series of sin and cos (1/n! coefficients) at h = y / 2 in [-pi/2, pi/2]
// (through h^13 / h^12, truncation below 7e-9) and the double-angle
// identities sin 2h = 2 sin h cos h, cos 2h = 1 - 2 sin^2 h (no quadrant
// selection, so nothing depends on k fitting an integer); in double, a table
// of sin and cos at multiples of pi / 64 and the short series of the
// remainder (see the function).
//
// rotate_small: (sin x, cos x) -> (sin(x+d), cos(x+d)) by angle addition with
// the series of sin d and cos d; used for |d| <= kRotMax, exact to rounding
// there (double: d^9/9! < 6e-18 at |d| = 0.05; float: see small_sc).
#pragma once

#include <hip/hip_runtime.h>

namespace sgp4mi {

constexpr double kRotMax = 0.05;

// Double-precision constants live in constant memory: gfx9 VALU instructions
// take no 64-bit literals, and scalar-register operands (one per instruction)
// avoid holding every coefficient in a vector register pair.
// The small-angle rotation reads its terms from indices 7-9 and 16-18; the
// other orders are kept for reference.
__constant__ double kHalfAngle64[24] = {
    // sin h = h + h^3 * P(h^2): -1/3!, 1/5!, ..., 1/21! (index 0 = highest order)
    1.95729410633912612308e-20, -8.22063524662432971696e-18, 2.8114572543455207632e-15,
    -7.6471637318198164759e-13, 1.60590438368216145994e-10, -2.50521083854417187751e-8,
    2.75573192239858906526e-6, -1.98412698412698412698e-4, 8.33333333333333333333e-3,
    -1.66666666666666666667e-1,
    // cos h = 1 + h^2 * Q(h^2): -1/2!, 1/4!, ..., 1/20! (index 10 = highest order)
    4.11031762331216485848e-19, -1.56192069685862264622e-16, 4.77947733238738529744e-14,
    -1.14707455977297247139e-11, 2.08767569878680989792e-9, -2.75573192239858906526e-7,
    2.48015873015873015873e-5, -1.38888888888888888889e-3, 4.16666666666666666667e-2, -0.5,
    // 1 / (2*pi), 2*pi (double nearest), 2*pi minus that
    0.15915494309189533577, 6.2831853071795864769, 2.4492935982947063e-16,
    // unused
    0.0};

__device__ __forceinline__ void half_angle(float h, float* s, float* c) {
  const float h2 = h * h;
  float p = fmaf(h2, 1.60590438368e-10f, -2.50521083854e-8f);
  p = fmaf(p, h2, 2.75573192240e-6f);
  p = fmaf(p, h2, -1.98412698413e-4f);
  p = fmaf(p, h2, 8.33333333333e-3f);
  p = fmaf(p, h2, -1.66666666667e-1f);
  const float sh = fmaf(p * h2, h, h);
  float q = fmaf(h2, 2.08767569879e-9f, -2.75573192240e-7f);
  q = fmaf(q, h2, 2.48015873016e-5f);
  q = fmaf(q, h2, -1.38888888889e-3f);
  q = fmaf(q, h2, 4.16666666667e-2f);
  q = fmaf(q, h2, -0.5f);
  const float ch = fmaf(q, h2, 1.0f);
  *s = 2.0f * sh * ch;
  *c = fmaf(-2.0f * sh, sh, 1.0f);
}

// sin and cos of j pi / 64 for j = -64 .. 64, interleaved (sin, cos), each the
// double nearest the exact value.
__constant__ double kSinCos64[258] = {
    0.0, -1.0, -0.049067674327418015, -0.9987954562051724,
    -0.0980171403295606, -0.9951847266721969, -0.14673047445536175, -0.989176509964781,
    -0.19509032201612828, -0.9807852804032304, -0.2429801799032639, -0.970031253194544,
    -0.2902846772544624, -0.9569403357322088, -0.33688985339222005, -0.9415440651830208,
    -0.3826834323650898, -0.9238795325112867, -0.4275550934302821, -0.9039892931234433,
    -0.47139673682599764, -0.881921264348355, -0.5141027441932218, -0.8577286100002721,
    -0.5555702330196022, -0.8314696123025452, -0.5956993044924334, -0.8032075314806449,
    -0.6343932841636455, -0.773010453362737, -0.6715589548470184, -0.7409511253549591,
    -0.7071067811865476, -0.7071067811865476, -0.7409511253549591, -0.6715589548470184,
    -0.773010453362737, -0.6343932841636455, -0.8032075314806449, -0.5956993044924334,
    -0.8314696123025452, -0.5555702330196022, -0.8577286100002721, -0.5141027441932218,
    -0.881921264348355, -0.47139673682599764, -0.9039892931234433, -0.4275550934302821,
    -0.9238795325112867, -0.3826834323650898, -0.9415440651830208, -0.33688985339222005,
    -0.9569403357322088, -0.2902846772544624, -0.970031253194544, -0.2429801799032639,
    -0.9807852804032304, -0.19509032201612828, -0.989176509964781, -0.14673047445536175,
    -0.9951847266721969, -0.0980171403295606, -0.9987954562051724, -0.049067674327418015,
    -1.0, 0.0, -0.9987954562051724, 0.049067674327418015,
    -0.9951847266721969, 0.0980171403295606, -0.989176509964781, 0.14673047445536175,
    -0.9807852804032304, 0.19509032201612828, -0.970031253194544, 0.2429801799032639,
    -0.9569403357322088, 0.2902846772544624, -0.9415440651830208, 0.33688985339222005,
    -0.9238795325112867, 0.3826834323650898, -0.9039892931234433, 0.4275550934302821,
    -0.881921264348355, 0.47139673682599764, -0.8577286100002721, 0.5141027441932218,
    -0.8314696123025452, 0.5555702330196022, -0.8032075314806449, 0.5956993044924334,
    -0.773010453362737, 0.6343932841636455, -0.7409511253549591, 0.6715589548470184,
    -0.7071067811865476, 0.7071067811865476, -0.6715589548470184, 0.7409511253549591,
    -0.6343932841636455, 0.773010453362737, -0.5956993044924334, 0.8032075314806449,
    -0.5555702330196022, 0.8314696123025452, -0.5141027441932218, 0.8577286100002721,
    -0.47139673682599764, 0.881921264348355, -0.4275550934302821, 0.9039892931234433,
    -0.3826834323650898, 0.9238795325112867, -0.33688985339222005, 0.9415440651830208,
    -0.2902846772544624, 0.9569403357322088, -0.2429801799032639, 0.970031253194544,
    -0.19509032201612828, 0.9807852804032304, -0.14673047445536175, 0.989176509964781,
    -0.0980171403295606, 0.9951847266721969, -0.049067674327418015, 0.9987954562051724,
    0.0, 1.0, 0.049067674327418015, 0.9987954562051724,
    0.0980171403295606, 0.9951847266721969, 0.14673047445536175, 0.989176509964781,
    0.19509032201612828, 0.9807852804032304, 0.2429801799032639, 0.970031253194544,
    0.2902846772544624, 0.9569403357322088, 0.33688985339222005, 0.9415440651830208,
    0.3826834323650898, 0.9238795325112867, 0.4275550934302821, 0.9039892931234433,
    0.47139673682599764, 0.881921264348355, 0.5141027441932218, 0.8577286100002721,
    0.5555702330196022, 0.8314696123025452, 0.5956993044924334, 0.8032075314806449,
    0.6343932841636455, 0.773010453362737, 0.6715589548470184, 0.7409511253549591,
    0.7071067811865476, 0.7071067811865476, 0.7409511253549591, 0.6715589548470184,
    0.773010453362737, 0.6343932841636455, 0.8032075314806449, 0.5956993044924334,
    0.8314696123025452, 0.5555702330196022, 0.8577286100002721, 0.5141027441932218,
    0.881921264348355, 0.47139673682599764, 0.9039892931234433, 0.4275550934302821,
    0.9238795325112867, 0.3826834323650898, 0.9415440651830208, 0.33688985339222005,
    0.9569403357322088, 0.2902846772544624, 0.970031253194544, 0.2429801799032639,
    0.9807852804032304, 0.19509032201612828, 0.989176509964781, 0.14673047445536175,
    0.9951847266721969, 0.0980171403295606, 0.9987954562051724, 0.049067674327418015,
    1.0, 0.0, 0.9987954562051724, -0.049067674327418015,
    0.9951847266721969, -0.0980171403295606, 0.989176509964781, -0.14673047445536175,
    0.9807852804032304, -0.19509032201612828, 0.970031253194544, -0.2429801799032639,
    0.9569403357322088, -0.2902846772544624, 0.9415440651830208, -0.33688985339222005,
    0.9238795325112867, -0.3826834323650898, 0.9039892931234433, -0.4275550934302821,
    0.881921264348355, -0.47139673682599764, 0.8577286100002721, -0.5141027441932218,
    0.8314696123025452, -0.5555702330196022, 0.8032075314806449, -0.5956993044924334,
    0.773010453362737, -0.6343932841636455, 0.7409511253549591, -0.6715589548470184,
    0.7071067811865476, -0.7071067811865476, 0.6715589548470184, -0.7409511253549591,
    0.6343932841636455, -0.773010453362737, 0.5956993044924334, -0.8032075314806449,
    0.5555702330196022, -0.8314696123025452, 0.5141027441932218, -0.8577286100002721,
    0.47139673682599764, -0.881921264348355, 0.4275550934302821, -0.9039892931234433,
    0.3826834323650898, -0.9238795325112867, 0.33688985339222005, -0.9415440651830208,
    0.2902846772544624, -0.9569403357322088, 0.2429801799032639, -0.970031253194544,
    0.19509032201612828, -0.9807852804032304, 0.14673047445536175, -0.989176509964781,
    0.0980171403295606, -0.9951847266721969, 0.049067674327418015, -0.9987954562051724,
    0.0, -1.0,
};

// A constant held in a scalar register.  gfx9 three-operand
// instructions take no literal, so a fused multiply-add with a literal factor
// and a second constant costs an extra vector move; with the factor in a
// scalar register (set by a scalar move) it is one instruction.
__device__ __forceinline__ float sgpr_const(float x) {
  asm("" : "+s"(x));
  return x;
}
__device__ __forceinline__ double sgpr_const(double x) {
  asm("" : "+s"(x));
  return x;
}

// Double: y = x - 2 pi n as above, then y = j pi / 64 + b with |b| <= pi / 128
// (a two-part pi / 64), the table's sin and cos of j pi / 64 and the series of
// sin b through b^7 and cos b through b^6 (the next terms are below 4e-19 and
// 3.3e-18 relative), combined by angle addition.  The table index is clamped,
// so no input (NaN, infinity, huge) reads outside the table.
__device__ __forceinline__ void sincos_rr(double x, double* s, double* c) {
  const double* k = kHalfAngle64;
  const double n = rint(x * k[20]);
  double y = fma(-n, k[21], x);
  y = fma(-n, k[22], y);
  const double jd = rint(y * 20.371832715762604);  // 64 / pi
  double b = fma(-jd, 0.04908738521234052, y);     // pi / 64, nearest double
  b = fma(-jd, 1.9135106236677394e-18, b);         // pi / 64 minus that
  int j = int(jd) + 64;
  j = j < 0 ? 0 : (j > 128 ? 128 : j);
  // The clamped index is non-negative: read the pair at a 32-bit byte offset
  // from the table's base, seen in the global address space (the load then
  // takes the base from scalar registers and needs no 64-bit address).
  uint32_t off = uint32_t(j) * 16u;
  asm("" : "+v"(off));
  typedef const __attribute__((address_space(1))) char* GBytes;
  typedef const __attribute__((address_space(1))) double* GDouble;
  const GDouble e = (GDouble)((GBytes)(const char*)kSinCos64 + off);
  const double sa = e[0], ca = e[1];
  const double b2 = b * b;
  // Coefficients in scalar registers (an instruction reads at most one); the
  // first step of each polynomial holds two of them, so it is a product and a
  // sum instead of a fused multiply-add that would need one moved into vector
  // registers first.
  double p, q;
  {
#pragma clang fp contract(off)
    p = b2 * sgpr_const(-1.98412698412698412698e-4) + sgpr_const(8.33333333333333333333e-3);
    q = b2 * sgpr_const(-1.38888888888888888889e-3) + sgpr_const(4.16666666666666666667e-2);
  }
  p = fma(p, b2, sgpr_const(-1.66666666666666666667e-1));
  const double sb = fma(p * b2, b, b);
  q = fma(q, b2, -0.5);
  const double cb = fma(q, b2, 1.0);
  *s = fma(sa, cb, ca * sb);
  *c = fma(ca, cb, -(sa * sb));
}

__device__ __forceinline__ void sincos_rr(float x, float* s, float* c) {
  const float n = rintf(x * 0.15915494309189533577f);
  float y = fmaf(-n, 6.28318548202514648438f, x);   // float nearest 2*pi
  y = fmaf(-n, -1.7484556e-7f, y);                   // 2*pi minus that
  half_angle(0.5f * y, s, c);
}

// Hardware sine and cosine (v_sin_f32 / v_cos_f32 take the argument in
// revolutions): the angle is reduced to a fraction of a turn in its own type,
// then rounded to float.
__device__ __forceinline__ void sincos_hw(double x, float* s, float* c) {
  const float r = float(__builtin_amdgcn_fract(x * kHalfAngle64[20]));
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void sincos_hw(float x, float* s, float* c) {
  const float r = __builtin_amdgcn_fractf(x * 0.15915494309189533577f);
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}

__device__ __forceinline__ void small_sc(double d, double* sd, double* cd) {
  const double* k = kHalfAngle64;
  const double d2 = d * d;
  double ps = fma(d2, k[7], k[8]);  // -1/7!, 1/5!
  ps = fma(ps, d2, k[9]);            // -1/3!
  *sd = fma(ps * d2, d, d);
  double pc = fma(d2, k[16], k[17]);  // 1/8!, -1/6!
  pc = fma(pc, d2, k[18]);            // 1/4!
  pc = fma(pc, d2, -0.5);
  *cd = fma(pc, d2, 1.0);
}

// Float: through d^3 (sine) and d^4 (cosine); the next terms are below
// 2.6e-9 and 2.2e-11 at |d| = 0.05, under the float rounding of the result.
__device__ __forceinline__ void small_sc(float d, float* sd, float* cd) {
  const float d2 = d * d;
  *sd = fmaf(d2 * d, -1.6666666667e-1f, d);
  float pc = fmaf(d2, sgpr_const(4.1666666667e-2f), -0.5f);
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

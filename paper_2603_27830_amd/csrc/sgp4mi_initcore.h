// Per-satellite initialisation of the near-Earth model, templated on the
// scalar so the same steps give the constant record (double) and its
// derivatives with respect to the elements (forward-mode Dual1) for the VJP.
//
// Steps of the published model the paper re-implements (section 2.1:
// Hoots & Roehrich 1980 / Hoots et al. 2004 / Vallado et al. 2006, WGS72):
// recovery of the original mean motion and semi-major axis from the element
// set's Kozai mean motion, the perigee-dependent atmospheric parameters, the
// power-law drag coefficients C1..C5 and D2..D4, the J2/J2^2/J4 secular rates
// and the J3 long-period coefficients.  The satellite-level validity checks
// (eccentricity at epoch, recovered mean motion, 225-minute deep-space
// boundary of section 6) are resolved here, once per satellite.
#pragma once

#include "sgp4mi_common.h"
#include "sgp4mi_math.h"

namespace sgp4mi {

// Forward-mode dual number with one tangent (value, derivative).  Kept in its
// own namespace so its math overloads are found by argument-dependent lookup
// only and never hide the double versions.
namespace dual {
struct Dual1 {
  double v, d;
  __device__ Dual1() : v(0), d(0) {}
  __device__ Dual1(double x) : v(x), d(0) {}  // NOLINT: constants promote implicitly
  __device__ Dual1(double x, double dx) : v(x), d(dx) {}
};
__device__ __forceinline__ double value(const Dual1& x) { return x.v; }
__device__ __forceinline__ Dual1 operator+(Dual1 a, Dual1 b) { return Dual1(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual1 operator-(Dual1 a, Dual1 b) { return Dual1(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual1 operator-(Dual1 a) { return Dual1(-a.v, -a.d); }
__device__ __forceinline__ Dual1 operator*(Dual1 a, Dual1 b) { return Dual1(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dual1 operator/(Dual1 a, Dual1 b) {
  const double q = a.v / b.v;
  return Dual1(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ Dual1 operator+(Dual1 a, double b) { return Dual1(a.v + b, a.d); }
__device__ __forceinline__ Dual1 operator+(double a, Dual1 b) { return Dual1(a + b.v, b.d); }
__device__ __forceinline__ Dual1 operator-(Dual1 a, double b) { return Dual1(a.v - b, a.d); }
__device__ __forceinline__ Dual1 operator-(double a, Dual1 b) { return Dual1(a - b.v, -b.d); }
__device__ __forceinline__ Dual1 operator*(Dual1 a, double b) { return Dual1(a.v * b, a.d * b); }
__device__ __forceinline__ Dual1 operator*(double a, Dual1 b) { return Dual1(a * b.v, a * b.d); }
__device__ __forceinline__ Dual1 operator/(Dual1 a, double b) { return Dual1(a.v / b, a.d / b); }
__device__ __forceinline__ Dual1 operator/(double a, Dual1 b) {
  const double q = a / b.v;
  return Dual1(q, -q * b.d / b.v);
}
__device__ __forceinline__ Dual1 sqrt(Dual1 x) {
  const double s = ::sqrt(x.v);
  return Dual1(s, 0.5 * x.d / s);
}
__device__ __forceinline__ Dual1 cbrt(Dual1 x) {
  const double c = ::cbrt(x.v);
  return Dual1(c, x.d / (3.0 * c * c));
}
__device__ __forceinline__ Dual1 fabs(Dual1 x) { return x.v < 0 ? -x : x; }
__device__ __forceinline__ void sin_cos(Dual1 x, Dual1* s, Dual1* c) {
  double sv, cv;
  sincos_rr(x.v, &sv, &cv);
  *s = Dual1(sv, cv * x.d);
  *c = Dual1(cv, -sv * x.d);
}

}  // namespace dual
using dual::Dual1;
__device__ __forceinline__ double value(double x) { return x; }
using dual::value;
// Sine and cosine of an element angle: the reduced-range series of the
// propagation kernels (any argument, no quadrant logic, no library branches).
__device__ __forceinline__ void sin_cos(double x, double* s, double* c) { sincos_rr(x, s, c); }
using dual::sin_cos;
// Quotient: for double, the reciprocal estimate refined by Newton steps times
// the numerator (within about an ulp of the rounded quotient, and a shorter
// dependency chain than the correctly rounded division); for dual numbers, their
// own division.
__device__ __forceinline__ double quot(double a, double b) { return a * rcp(b); }
template <class A, class B>
__device__ __forceinline__ Dual1 quot(A a, B b) { return Dual1(a) / Dual1(b); }

struct GravIn {
  double radius, j2, j4, ke, j3oj2;
};

// el: n0 (Kozai, rad/min), e0, i0, node0, argp0, M0, bstar.  Writes the
// record entries (all but kEpochMin), the satellite code and the flag.
template <class S>
__device__ __forceinline__ void init_record(const GravIn& g, const S el[7], S rec[kNRec], uint32_t* code_out,
                                            bool* isimp_out) {
  using ::cbrt;
  using ::fabs;
  using ::sqrt;
  const S& no_kozai = el[0];
  const S& ecco = el[1];
  const S& inclo = el[2];
  const S& nodeo = el[3];
  const S& argpo = el[4];
  const S& mo = el[5];
  const S& bstar = el[6];
  const double R = g.radius, J2 = g.j2, J4 = g.j4, ke = g.ke, j3oj2 = g.j3oj2;

  S sin_i, cos_i;
  sin_cos(inclo, &sin_i, &cos_i);
  const S c2 = cos_i * cos_i;
  const S omeosq = 1.0 - ecco * ecco;  // beta0^2
  const S rteosq = sqrt(omeosq);       // beta0
  const S con41 = 3.0 * c2 - 1.0;
  const S x1mth2 = 1.0 - c2;
  const S x7thm1 = 7.0 * c2 - 1.0;

  // Original mean motion: invert the Kozai definition with the second-order
  // correction of the published model.
  const S ak = cbrt(quot(ke, no_kozai));
  const S a1 = ak * ak;
  const S d1 = quot(0.75 * J2 * con41, rteosq * omeosq);
  const S del1 = quot(d1, a1 * a1);
  const S adel = a1 * (1.0 - del1 * (1.0 / 3.0 + del1 * (1.0 + (134.0 / 81.0) * del1)));
  const S del0 = quot(d1, adel * adel);
  const S nbar = quot(no_kozai, 1.0 + del0);
  const S ab = cbrt(quot(ke, nbar));
  const S abar = ab * ab;

  // Perigee height -> density parameter s and (q0 - s)^4.
  const S perigee_er = abar * (1.0 - ecco);
  const S perigee_km = (perigee_er - 1.0) * R;
  S sfour = S(1.0 + 78.0 / R);
  S qoms = S((120.0 - 78.0) / R);
  if (value(perigee_km) < 156.0) {
    const S s_km = (value(perigee_km) < 98.0) ? S(20.0) : perigee_km - 78.0;
    qoms = (120.0 - s_km) / R;
    sfour = 1.0 + s_km / R;
  }
  const S qoms2 = qoms * qoms;
  const S qoms24 = qoms2 * qoms2;

  const bool isimp = value(perigee_er) < 1.0 + 220.0 / R;
  uint32_t code = 0;
  if (!(value(ecco) >= 0.0 && value(ecco) < 1.0)) code = 1;
  else if (!(value(nbar) > 0.0)) code = 2;
  else if (kTwoPi / value(nbar) >= 225.0) code = 7;

  // Power-law drag coefficients.
  const S tsi = quot(1.0, abar - sfour);
  const S eta = abar * ecco * tsi;
  const S etasq = eta * eta;
  const S eeta = ecco * eta;
  const S psisq = fabs(1.0 - etasq);
  const S tsi2 = tsi * tsi;
  const S coef = qoms24 * tsi2 * tsi2;
  const S coef1 = quot(coef, psisq * psisq * psisq * sqrt(psisq));
  const S cc2 = coef1 * nbar *
                (abar * (1.0 + 1.5 * etasq + eeta * (4.0 + etasq)) +
                 0.375 * J2 * quot(tsi, psisq) * con41 * (8.0 + 3.0 * etasq * (8.0 + etasq)));
  const S cc1 = bstar * cc2;
  const S cc3 = (value(ecco) > 1.0e-4) ? quot(-2.0 * coef * tsi * j3oj2 * nbar * sin_i, ecco) : S(0.0);
  S sin_w, cos_w;
  sin_cos(argpo, &sin_w, &cos_w);
  const S cos_2w = 2.0 * cos_w * cos_w - 1.0;
  const S cc4 = 2.0 * nbar * coef1 * abar * omeosq *
                (eta * (2.0 + 0.5 * etasq) + ecco * (0.5 + 2.0 * etasq) -
                 quot(J2 * tsi, abar * psisq) *
                     (-3.0 * con41 * (1.0 - 2.0 * eeta + etasq * (1.5 - 0.5 * eeta)) +
                      0.75 * x1mth2 * (2.0 * etasq - eeta * (1.0 + etasq)) * cos_2w));
  const S cc5 = 2.0 * coef1 * abar * omeosq * (1.0 + 2.75 * (etasq + eeta) + eeta * etasq);

  // Secular rates.
  const S pinv = quot(1.0, abar * omeosq);
  const S pinvsq = pinv * pinv;
  const S c4 = c2 * c2;
  const S temp1 = 1.5 * J2 * pinvsq * nbar;
  const S temp2 = 0.5 * temp1 * J2 * pinvsq;
  const S temp3 = -0.46875 * J4 * pinvsq * pinvsq * nbar;
  const S mdot = nbar + 0.5 * temp1 * rteosq * con41 + 0.0625 * temp2 * rteosq * (13.0 - 78.0 * c2 + 137.0 * c4);
  const S argpdot = -0.5 * temp1 * (1.0 - 5.0 * c2) + 0.0625 * temp2 * (7.0 - 114.0 * c2 + 395.0 * c4) +
                    temp3 * (3.0 - 36.0 * c2 + 49.0 * c4);
  const S xhdot1 = -temp1 * cos_i;
  const S nodedot = xhdot1 + (0.5 * temp2 * (4.0 - 19.0 * c2) + 2.0 * temp3 * (3.0 - 7.0 * c2)) * cos_i;

  S sin_m0, cos_m0;
  sin_cos(mo, &sin_m0, &cos_m0);
  S argpcof = bstar * cc3 * cos_w;
  S xmcof = (value(ecco) > 1.0e-4) ? quot(-(2.0 / 3.0) * coef * bstar, eeta) : S(0.0);
  const S nodecf = 3.5 * omeosq * xhdot1 * cc1;
  const S t2cof = 1.5 * cc1;
  S den = 1.0 + cos_i;
  if (::fabs(value(den)) <= 1.5e-12) den = S(1.5e-12);
  const S xlcof = quot(-0.25 * j3oj2 * sin_i * (3.0 + 5.0 * cos_i), den);
  const S aycof = -0.5 * j3oj2 * sin_i;
  const S dm = 1.0 + eta * cos_m0;
  const S delmo = dm * dm * dm;

  S d2 = S(0.0), d3 = S(0.0), d4 = S(0.0), t3cof = S(0.0), t4cof = S(0.0), t5cof = S(0.0);
  S bc5 = bstar * cc5;
  if (!isimp) {
    const S cc1sq = cc1 * cc1;
    d2 = 4.0 * abar * tsi * cc1sq;
    const S tmp = d2 * tsi * cc1 * (1.0 / 3.0);
    d3 = (17.0 * abar + sfour) * tmp;
    d4 = 0.5 * tmp * abar * tsi * (221.0 * abar + 31.0 * sfour) * cc1;
    t3cof = d2 + 2.0 * cc1sq;
    t4cof = 0.25 * (3.0 * d3 + cc1 * (12.0 * d2 + 10.0 * cc1sq));
    t5cof = 0.2 * (3.0 * d4 + 12.0 * cc1 * d3 + 6.0 * d2 * d2 + 15.0 * cc1sq * (2.0 * d2 + cc1sq));
  } else {
    // The simplified model applies none of these; zeroing them makes the
    // general per-point expression reduce exactly to the simplified one.
    argpcof = S(0.0);
    xmcof = S(0.0);
    bc5 = S(0.0);
  }

  rec[kM0] = mo; rec[kMdot] = mdot; rec[kArgp0] = argpo; rec[kArgpdot] = argpdot;
  rec[kNode0] = nodeo; rec[kNodedot] = nodedot; rec[kNodecf] = nodecf; rec[kC1] = cc1;
  rec[kBC4] = bstar * cc4; rec[kT2cof] = t2cof; rec[kArgpcof] = argpcof; rec[kEta] = eta;
  rec[kMcof] = xmcof; rec[kDM0] = delmo; rec[kD2] = d2; rec[kD3] = d3; rec[kD4] = d4;
  rec[kBC5] = bc5; rec[kSinM0] = sin_m0; rec[kT3cof] = t3cof; rec[kT4cof] = t4cof; rec[kT5cof] = t5cof;
  rec[kN0pp] = nbar; rec[kA0pp] = abar; rec[kE0] = ecco; rec[kAycof] = aycof; rec[kLcof] = xlcof;
  rec[kC41] = con41; rec[kX1] = x1mth2; rec[kX7] = x7thm1; rec[kCosi] = cos_i; rec[kSini] = sin_i;
  rec[kI0] = inclo;
  rec[kEpochMin] = S(0.0);
  *code_out = code;
  *isimp_out = isimp;
}

}  // namespace sgp4mi

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
// record entries (all but kEpochMin), the satellite code and the flags
// (simplified drag; deep space: period of 225 min or more, which also takes
// the simplified drag terms).
template <class S>
__device__ __forceinline__ void init_record(const GravIn& g, const S el[7], S rec[kNRec], uint32_t* code_out,
                                            bool* isimp_out, bool* deep_out) {
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

  uint32_t code = 0;
  bool deep = false;
  if (!(value(ecco) >= 0.0 && value(ecco) < 1.0)) code = 1;
  else if (!(value(nbar) > 0.0)) code = 2;
  else if (kTwoPi / value(nbar) >= 225.0) deep = true;
  const bool isimp = deep || value(perigee_er) < 1.0 + 220.0 / R;

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
  const double k2 = 0.5 * J2;
  rec[kSpA1] = (1.5 * k2) * con41; rec[kSpX1h] = (0.5 * k2) * x1mth2; rec[kSpX1k] = k2 * x1mth2;
  rec[kSpX7q] = (-0.25 * k2) * x7thm1; rec[kSpCN] = (1.5 * k2) * cos_i; rec[kSpCI] = (1.5 * k2) * cos_i * sin_i;
  *code_out = code;
  *isimp_out = isimp;
  *deep_out = deep;
}

// ---------------------------------------------------------- deep space --
// Lunar-solar part of the deep-space initialisation (Hujsak's terms in the
// published model): from the satellite's epoch elements and the absolute
// epoch, the secular rates and the long-period coefficients of the Sun's and
// the Moon's quadrupole tidal potential, each averaged over the satellite's
// orbit, and the two bodies' mean anomalies at epoch.  Double precision, one
// lane per satellite.  day: epoch in days after JD 2415020.0.
struct DeepBody {
  double n, e, c1;  // mean motion (rad/min), orbit eccentricity, tidal strength / (4 n)
};
constexpr DeepBody kSun{1.19459e-5, 0.01675, 2.9864797e-6};
constexpr DeepBody kMoon{1.5835218e-4, 0.05490, 4.7968065e-7};

// Coefficients of one body whose orbit has perigee argument g (from its node
// on the equator), inclination ib to the equator, and whose node lies h
// before the satellite's node (cos/sin of each), for a satellite of
// inclination i, perigee argument w, eccentricity e, mean motion n.  out: the
// kNPer long-period coefficients; sec: the body's contributions to the rates
// of e, i, M, argp + cos i node and sin i node (before the division by sin i).
__device__ inline void deep_body(double cg, double sg, double cib, double sib, double ch, double sh, double cw,
                                 double sw, double ci, double si, double e, double n, const DeepBody& b,
                                 double* out, double sec[5]) {
  const double e2 = e * e, beta2 = 1.0 - e2, beta = sqrt(beta2);
  // body perigee (p) and its normal-plane axis (q) projected on the
  // satellite's node line, its in-plane normal and its orbit pole
  const double p1 = cg * ch + sg * cib * sh;
  const double q1 = -sg * ch + cg * cib * sh;
  const double pn = -cg * sh + sg * cib * ch;
  const double qn = sg * sh + cg * cib * ch;
  const double p2 = ci * pn + si * sg * sib;
  const double q2 = ci * qn + si * cg * sib;
  const double p3 = -si * pn + ci * sg * sib;
  const double q3 = -si * qn + ci * cg * sib;
  // ... then on the satellite's perigee direction (x*) and the direction a
  // quarter turn ahead (y*); the pole components take sin w and cos w
  const double xp = p1 * cw + p2 * sw, xq = q1 * cw + q2 * sw;
  const double yp = -p1 * sw + p2 * cw, yq = -q1 * sw + q2 * cw;
  const double zps = p3 * sw, zqs = q3 * sw, zpc = p3 * cw, zqc = q3 * cw;
  const double zz1 = 12.0 * xp * xp - 3.0 * yp * yp;
  const double zz2 = 24.0 * xp * xq - 6.0 * yp * yq;
  const double zz3 = 12.0 * xq * xq - 3.0 * yq * yq;
  const double z1 = 2.0 * (3.0 * (p1 * p1 + p2 * p2) + zz1 * e2) + beta2 * zz1;
  const double z2 = 2.0 * (6.0 * (p1 * q1 + p2 * q2) + zz2 * e2) + beta2 * zz2;
  const double z3 = 2.0 * (3.0 * (q1 * q1 + q2 * q2) + zz3 * e2) + beta2 * zz3;
  const double z11 = -6.0 * p1 * p3 + e2 * (-24.0 * xp * zpc - 6.0 * yp * zps);
  const double z12 = -6.0 * (p1 * q3 + q1 * p3) + e2 * (-24.0 * (xq * zpc + xp * zqc) - 6.0 * (yp * zqs + yq * zps));
  const double z13 = -6.0 * q1 * q3 + e2 * (-24.0 * xq * zqc - 6.0 * yq * zqs);
  const double z21 = 6.0 * p2 * p3 + e2 * (24.0 * xp * zps - 6.0 * yp * zpc);
  const double z22 = 6.0 * (q2 * p3 + p2 * q3) + e2 * (24.0 * (xq * zps + xp * zqs) - 6.0 * (yq * zpc + yp * zqc));
  const double z23 = 6.0 * q2 * q3 + e2 * (24.0 * xq * zqs - 6.0 * yq * zqc);
  const double s3 = b.c1 / n;
  const double s2 = -0.5 * s3 / beta;
  const double s4 = s3 * beta;
  const double s1 = -15.0 * e * s4;
  const double s5 = xp * yp + xq * yq;
  const double s6 = xq * yp + xp * yq;
  const double s7 = xq * yq - xp * yp;
  out[kPe2] = 2.0 * s1 * s6;
  out[kPe3] = 2.0 * s1 * s7;
  out[kPi2] = 2.0 * s2 * z12;
  out[kPi3] = 2.0 * s2 * (z13 - z11);
  out[kPl2] = -2.0 * s3 * z2;
  out[kPl3] = -2.0 * s3 * (z3 - z1);
  out[kPl4] = -2.0 * s3 * (-21.0 - 9.0 * e2) * b.e;
  out[kPgh2] = 2.0 * s4 * zz2;
  out[kPgh3] = 2.0 * s4 * (zz3 - zz1);
  out[kPgh4] = -18.0 * s4 * b.e;
  out[kPh2] = -2.0 * s2 * z22;
  out[kPh3] = -2.0 * s2 * (z23 - z21);
  sec[0] = s1 * b.n * s5;
  sec[1] = s2 * b.n * (z11 + z13);
  sec[2] = -b.n * s3 * (z1 + z3 - 14.0 - 6.0 * e2);
  sec[3] = s4 * b.n * (zz1 + zz3 - 6.0);
  sec[4] = -b.n * s2 * (z21 + z23);
}

// ------------------------------------------------------------ resonance --
// Tesseral resonance (the published model's 24 h and 12 h classes): an
// orbit commensurate with the Earth's rotation feels the tesseral harmonics
// J_lm secularly through the arguments psi = j w + k lambda - phase, lambda
// the resonant mean longitude (24 h: M + node + w - theta, j = 0, k = m;
// 12 h: M + 2 node - 2 theta, j = l - 2p, k = m / 2); per term
// dn/dt = c sin psi with c = 3 n^2 (R/a)^l k J_lm F_lmp(i) G_lpq(e).

// Greenwich mean sidereal time (IAU 1982) of a Julian date taken as UT1,
// given as days after JD 2415020.0; radians in [0, 2 pi).
__device__ inline double gmst1982(double day) {
  const double T = (day - 36525.0) * (1.0 / 36525.0);
  const double sec = 67310.54841 + T * ((876600.0 * 3600.0 + 8640184.812866) + T * (0.093104 - 6.2e-6 * T));
  const double x = fmod(sec, 86400.0) * (kTwoPi / 86400.0);
  return x < 0.0 ? x + kTwoPi : x;
}

// Per-satellite resonance terms.  rec: the satellite's record (mean motion,
// inclination functions, secular rates); d: its deep-space slot with the
// lunar-solar rates already written; M0, node0, argp0, e0 from el.
__device__ inline void init_resonance(const double el[7], const double* rec, double ke, double day, double* d) {
  const double n = rec[kN0pp], e = el[1];
  const int cls = (n < 0.0052359877 && n > 0.0034906585) ? 1 : (n >= 8.26e-3 && n <= 9.24e-3 && e >= 0.5) ? 2 : 0;
  const double gsto = gmst1982(day);
  d[kDRes] = double(cls);
  d[kDGsto] = gsto;
  d[kDXlamo] = 0.0;
  d[kDXfact] = 0.0;
#pragma unroll
  for (int m = 0; m < 20; ++m) d[kDRc0 + m] = 0.0;
  if (cls == 0) return;
  const double ci = rec[kCosi], si = rec[kSini], c2 = ci * ci, s2 = si * si;
  const double ra = cbrt(n / ke) * cbrt(n / ke);  // R / a
  const double n2 = 3.0 * n * n * ra * ra;         // 3 n^2 (R/a)^2
  const double e2 = e * e, e3 = e2 * e;
  const double f220 = 0.75 * (1.0 + ci) * (1.0 + ci);
  // (k J F G (R/a)^(l-2), phase) per term
  double cf[10], ph[10];
  int nt;
  if (cls == 1) {
    // (l, m, p, q) = (3,1,1,0), (2,2,0,0), (3,3,0,0): F311 G310, F220 G200, F330 G300
    const double f311 = 0.9375 * s2 * (1.0 + 3.0 * ci) - 0.75 * (1.0 + ci);
    const double f330 = 1.875 * (1.0 + ci) * (1.0 + ci) * (1.0 + ci);
    const double g310 = 1.0 + 2.0 * e2;
    const double g200 = 1.0 + e2 * (-2.5 + 0.8125 * e2);
    const double g300 = 1.0 + e2 * (-6.0 + 6.60937 * e2);
    cf[0] = 2.1460748e-6 * f311 * g310 * ra;
    cf[1] = 2.0 * 1.7891679e-6 * f220 * g200;
    cf[2] = 3.0 * 2.2123015e-7 * f330 * g300 * ra;
    ph[0] = 0.13130908;
    ph[1] = 2.0 * 2.8843198;
    ph[2] = 3.0 * 0.37448087;
    nt = 3;
    d[kDXlamo] = el[5] + el[3] + el[4] - gsto;
    d[kDXfact] = rec[kMdot] + (rec[kArgpdot] + rec[kNodedot]) - kEarthRot + d[kDMDt] + d[kDArgpDt] + d[kDNodeDt] - n;
  } else {
    // Kaula's inclination functions of the ten terms
    const double f221 = 1.5 * s2;
    const double f321 = 1.875 * si * (1.0 - 2.0 * ci - 3.0 * c2);
    const double f322 = -1.875 * si * (1.0 + 2.0 * ci - 3.0 * c2);
    const double f441 = 35.0 * s2 * f220;
    const double f442 = 39.375 * s2 * s2;
    const double f522 = 9.84375 * si * (s2 * (1.0 - 2.0 * ci - 5.0 * c2) + 0.33333333 * (-2.0 + 4.0 * ci + 6.0 * c2));
    const double f523 = si * (4.92187512 * s2 * (-2.0 - 4.0 * ci + 10.0 * c2) + 6.56250012 * (1.0 + 2.0 * ci - 3.0 * c2));
    const double f542 = 29.53125 * si * (2.0 - 8.0 * ci + c2 * (-12.0 + 8.0 * ci + 10.0 * c2));
    const double f543 = 29.53125 * si * (-2.0 - 8.0 * ci + c2 * (12.0 + 8.0 * ci - 10.0 * c2));
    // the model's fits of the eccentricity functions over e >= 0.5
    const double g201 = -0.306 - (e - 0.64) * 0.440;
    double g211, g310, g322, g410, g422, g520, g533, g521, g532;
    if (e <= 0.65) {
      g211 = 3.616 - 13.2470 * e + 16.2900 * e2;
      g310 = -19.302 + 117.3900 * e - 228.4190 * e2 + 156.5910 * e3;
      g322 = -18.9068 + 109.7927 * e - 214.6334 * e2 + 146.5816 * e3;
      g410 = -41.122 + 242.6940 * e - 471.0940 * e2 + 313.9530 * e3;
      g422 = -146.407 + 841.8800 * e - 1629.014 * e2 + 1083.4350 * e3;
      g520 = -532.114 + 3017.977 * e - 5740.032 * e2 + 3708.2760 * e3;
    } else {
      g211 = -72.099 + 331.819 * e - 508.738 * e2 + 266.724 * e3;
      g310 = -346.844 + 1582.851 * e - 2415.925 * e2 + 1246.113 * e3;
      g322 = -342.585 + 1554.908 * e - 2366.899 * e2 + 1215.972 * e3;
      g410 = -1052.797 + 4758.686 * e - 7193.992 * e2 + 3651.957 * e3;
      g422 = -3581.690 + 16178.110 * e - 24462.770 * e2 + 12422.520 * e3;
      g520 = e > 0.715 ? -5149.66 + 29936.92 * e - 54087.36 * e2 + 31324.56 * e3
                       : 1464.74 - 4664.75 * e + 3763.64 * e2;
    }
    if (e < 0.7) {
      g533 = -919.22770 + 4988.6100 * e - 9064.7700 * e2 + 5542.21 * e3;
      g521 = -822.71072 + 4568.6173 * e - 8491.4146 * e2 + 5337.524 * e3;
      g532 = -853.66600 + 4690.2500 * e - 8624.7700 * e2 + 5341.4 * e3;
    } else {
      g533 = -37995.780 + 161616.52 * e - 229838.20 * e2 + 109377.94 * e3;
      g521 = -51752.104 + 218913.95 * e - 309468.16 * e2 + 146349.42 * e3;
      g532 = -40023.880 + 170470.89 * e - 242699.48 * e2 + 115605.82 * e3;
    }
    // (l m p q) = 2201 2211 3210 3222 4410 4422 5220 5232 5421 5433: J_lm,
    // phase m lambda_lm, k (1 or 2) and (R/a)^(l-2)
    const double ra2 = ra * ra, ra3 = ra2 * ra;
    cf[0] = 1.7891679e-6 * f220 * g201;
    cf[1] = 1.7891679e-6 * f221 * g211;
    cf[2] = 3.7393792e-7 * f321 * g310 * ra;
    cf[3] = 3.7393792e-7 * f322 * g322 * ra;
    cf[4] = 2.0 * 7.3636953e-9 * f441 * g410 * ra2;
    cf[5] = 2.0 * 7.3636953e-9 * f442 * g422 * ra2;
    cf[6] = 1.1428639e-7 * f522 * g520 * ra3;
    cf[7] = 1.1428639e-7 * f523 * g532 * ra3;
    cf[8] = 2.0 * 2.1765803e-9 * f542 * g521 * ra3;
    cf[9] = 2.0 * 2.1765803e-9 * f543 * g533 * ra3;
    ph[0] = ph[1] = 5.7686396;
    ph[2] = ph[3] = 0.95240898;
    ph[4] = ph[5] = 1.8014998;
    ph[6] = ph[7] = 1.0508330;
    ph[8] = ph[9] = 4.4108898;
    nt = 10;
    d[kDXlamo] = el[5] + 2.0 * el[3] - 2.0 * gsto;
    d[kDXfact] = rec[kMdot] + d[kDMDt] + 2.0 * (rec[kNodedot] + d[kDNodeDt] - kEarthRot) - n;
  }
  d[kDXlamo] = d[kDXlamo] - kTwoPi * floor(d[kDXlamo] * kInvTwoPi);
  for (int m = 0; m < nt; ++m) {
    double sp, cp;
    sincos_rr(ph[m], &sp, &cp);
    const double c = n2 * cf[m];
    d[kDRc0 + 2 * m] = c * cp;
    d[kDRc0 + 2 * m + 1] = c * sp;
  }
}

// el: epoch elements as for init_record; rec: the satellite's record (its
// recovered mean motion, inclination functions and secular rates); ke: the
// gravity's ke; day: days after JD 2415020.0.  Writes the kNDeep entries of a
// deep-space slot.
__device__ inline void init_deep(const double el[7], const double* rec, double ke, double day, double* d) {
  const double n = rec[kN0pp];
  const double e = el[1], inc = el[2];
  double si, ci, sw, cw, snd, cnd;
  sincos_rr(inc, &si, &ci);
  sincos_rr(el[4], &sw, &cw);
  sincos_rr(el[3], &snd, &cnd);
  // The Moon's orbit at epoch: node on the ecliptic, its inclination and node
  // on the equator (spherical triangle with the obliquity), its perigee
  // argument measured from that equatorial node.
  const double sin_eps = 0.39785416, cos_eps = 0.91744867, sin_il = 0.089683511;
  const double node_l = 4.5236020 - 9.2422029e-4 * day;
  double sl, cl;
  sincos_rr(node_l, &sl, &cl);
  const double cib_m = 0.91375164 - 0.03568096 * cl;
  const double sib_m = sqrt(1.0 - cib_m * cib_m);
  const double sh_l = sin_il * sl / sib_m;
  const double ch_l = sqrt(1.0 - sh_l * sh_l);
  const double perigee_l = 5.8351514 + 0.0019443680 * day;
  const double g_m = perigee_l + atan2(sin_eps * sl / sib_m, ch_l * cl + cos_eps * sh_l * sl) - node_l;
  double sg_m, cg_m;
  sincos_rr(g_m, &sg_m, &cg_m);
  double sec_s[5], sec_m[5];
  // Sun: node at the equinox, inclination the obliquity, perigee at 281.22 deg
  deep_body(0.1945905, -0.98088458, cos_eps, sin_eps, cnd, snd, cw, sw, ci, si, e, n, kSun, d + kDPer0, sec_s);
  deep_body(cg_m, sg_m, cib_m, sib_m, ch_l * cnd + sh_l * snd, snd * ch_l - cnd * sh_l, cw, sw, ci, si, e, n, kMoon,
            d + kDPer0 + kNPer, sec_m);
  // Satellite within 3 degrees of the equator: no lunar-solar node rate.
  const bool flat = inc < 5.2359877e-2 || inc > kPi - 5.2359877e-2;
  const double h = flat ? 0.0 : sec_s[4] + sec_m[4];
  const double dnode = si != 0.0 ? h / si : h;
  d[kDeDt] = sec_s[0] + sec_m[0];
  d[kDiDt] = sec_s[1] + sec_m[1];
  d[kDMDt] = sec_s[2] + sec_m[2];
  d[kDNodeDt] = dnode;
  d[kDArgpDt] = sec_s[3] + sec_m[3] - ci * dnode;
  const double ms = 6.2565837 + 0.017201977 * day;
  const double mm = 4.7199672 + 0.22997150 * day - perigee_l;
  d[kDMb0] = ms - kTwoPi * floor(ms * kInvTwoPi);
  d[kDMb1] = mm - kTwoPi * floor(mm * kInvTwoPi);
  init_resonance(el, rec, ke, day, d);
}

}  // namespace sgp4mi

// SGP4 near-Earth oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
//
// A plain, serial, double-precision CPU implementation of what the GPU library
// computes.  Only the test suite, the smoke check and the CPU-baseline leg of
// the benchmark may load it; the product library never links, calls or falls
// back to it, and the two share no source, header, table or helper.
//
// What it computes.  The paper (jaxsgp4, section 2.1 "Architecture and
// Refactoring") re-implements the SGP4 general-perturbation model of Hoots &
// Roehrich (Spacetrack Report No. 3, 1980) as revised by Hoots et al. (2004)
// and Vallado et al. (2006, AIAA 2006-6753), with the WGS72 geopotential
// constants, mapping a satellite's mean elements s and a time t to a TEME
// state f(s, t) -> (r, v) (section 2.2, "Vectorisation").  The paper prints
// none of the model's equations; the steps below restate the published
// near-Earth model in the order it is defined (initialisation I1-I8, then
// propagation P1-P9), written here from the mathematics, not from any listing.
// Orbits with periods of 225 min or more take the deep-space model's lunar and
// solar terms (Hujsak 1979 in the same reports; section 6 of the paper names
// deep space as the variant it leaves out): secular rates and long-period terms
// of the quadrupole tidal potential of the Sun and the Moon (I9, P2d, P4d), and,
// for the 12 h and 24 h resonant classes, the tesseral resonance of the
// geopotential, integrated in mean motion and mean longitude (I10, P3r).
//
// Readings where the paper is silent (each is listed in the design notes):
//  * WGS72: mu = 398600.8 km^3/s^2, R = 6378.135 km, J2 = 0.001082616,
//    J3 = -0.00000253881, J4 = -0.00000165597; ke = 60/sqrt(R^3/mu) 1/min.
//  * Un-Kozai'd semi-major axis a0'' = (ke/n0'')^(2/3) (Vallado 2006 form).
//  * Kepler: Newton on the generalised equation, start psi = U, step clamped to
//    [-0.95, 0.95], stop after the first step with |step| < 1e-12 or after 10
//    steps; sin/cos are then taken at the final iterate (the root).
//  * Error codes (section 2.2 "Control Flow": anomalous states are computed and
//    flagged, not exited): 1 mean eccentricity outside [-0.001, 1) (or e0
//    outside [0, 1) at epoch), 2 mean motion n0'' not > 0, 3 deep space: the
//    lunar-solar terms move e outside [0, 1], 4 semi-latus rectum p_L < 0, 6
//    decayed (r_k < 1 earth radius; state still written).  Checks run in the
//    order 1(epoch) -> 2 -> 2 (resonance-integrated mean motion) -> 1 -> 3 ->
//    4 -> 6; the first failing one wins.  Codes 1, 2, 3, 4 write NaN to r and v.
//    (Code 7, "not propagated", is the library's, for paths that leave deep
//    space out; this oracle never returns it.)
//  * Deep space: the lunar and solar arguments use absolute time, the epoch
//    row taken as days after a reference Julian date (J2000.0 unless set); the
//    node is reduced with floor to [0, 2*pi) before the low-inclination form
//    uses its value.  The Greenwich sidereal angle of the resonance is the
//    IAU 1982 mean sidereal time of that instant, taken as UT1.
//  * Checks are written so that NaN fails them (NaN never passes as valid).
//  * Angles are reduced with floor to [0, 2*pi).
//  * pow(x, 2/3) is cbrt(x)^2 and x^1.5 is x*sqrt(x).
//  * J3/J2 is taken as 0 when J3 == 0 (two-body configuration); J3 != 0 with
//    J2 == 0 is rejected.
//
// What pins it (CPU tests, each against something other than this file): the
// two-body closed form, node equivariance, Kepler residuals, finite
// differences, radius bounds, first-order J2 rates and Brouwer's second-order
// (J2^2) secular rates in the near-circular limit, the J2 field integrated over
// one orbit and the node over days, Lagrange's equations for the J4 rates and
// the J3 long-period terms, the drag coefficients as the power-law decay series
// and as Gauss-equation orbit averages (C2, C4, C5, the periodic drag term of M
// and w, the J3-drag perigee rate), the node drag term along the decaying
// orbit, the mean elements at epoch, term-group toggles, crafted error codes
// and a hand count of the operations.  Deep space: the lunar-solar constants
// against textbook astronomy, the five secular rates and the ten twice-anomaly
// periodic coefficients per body against Lagrange's equations on the
// numerically averaged quadrupole, the body-eccentricity terms, the
// low-inclination form at its switch, the resonance flags and code 3;
// resonance: the inclination functions against Kaula's closed form, the
// eccentricity functions against Hansen coefficients by quadrature, the 24 h
// rates against the tesseral field's along-track force on a geostationary
// orbit (stable longitudes, drift acceleration), the 12 h rates against the
// resonant arguments the tesseral terms select, the integrator against a
// fine numerical solution of its own equations, the sidereal time against
// its epoch value and rate, and a geostationary satellite's Earth-fixed
// longitude drift end to end.
//
// Parity unpinned (model definitions no available pin reaches): the J2 bracket
// of C4, the eccentricity factor (beta0^2) of the drag node term, the
// low-perigee density parameter (156 km / 98 km branch), the 220 km
// simplified-drag switch, the e0 > 1e-4 gate and the 1.5e-12 guard; in deep
// space the 0.2 rad switch value, the 3-degree cut of the node rate, the
// resonance bands, the first-order true anomaly of the bodies, the tesseral
// magnitudes and phases of degrees 3 to 5 of the 12 h class, the 720-minute
// step and the eccentricity ranges of the 12 h fits; and, as a
// whole, numeric agreement with the published model's own verification
// vectors, which are not available here.
//
// The scalar type is a template parameter: double for values, Dual (seven
// forward-mode tangents) for the derivative oracle, OpCount to count the
// arithmetic the definition performs.  Build: g++ -O2 -std=c++17
// -ffp-contract=off (no fast-math, no fused multiply-add contraction).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>
#include <algorithm>

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;
constexpr int kNElem = 7;  // differentiated elements: n0, e0, i0, node0, argp0, M0, bstar

// ---------------------------------------------------------------- scalars --
inline double val(double x) { return x; }

// Forward-mode dual number carrying derivatives w.r.t. the seven elements.
struct Dual {
  double v;
  double d[kNElem];
  Dual() : v(0) { std::memset(d, 0, sizeof d); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof d); }  // NOLINT: implicit by design
};
inline double val(const Dual& x) { return x.v; }
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int k = 0; k < kNElem; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int k = 0; k < kNElem; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int k = 0; k < kNElem; ++k) r.d[k] = -a.d[k]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int k = 0; k < kNElem; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int k = 0; k < kNElem; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int k = 0; k < kNElem; ++k) r.d[k] = a.d[k] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { Dual r(a.v / b); for (int k = 0; k < kNElem; ++k) r.d[k] = a.d[k] / b; return r; }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual chain(const Dual& x, double fx, double dfx) { Dual r(fx); for (int k = 0; k < kNElem; ++k) r.d[k] = dfx * x.d[k]; return r; }
inline Dual sin(const Dual& x) { return chain(x, std::sin(x.v), std::cos(x.v)); }
inline Dual cos(const Dual& x) { return chain(x, std::cos(x.v), -std::sin(x.v)); }
inline Dual sqrt(const Dual& x) { double s = std::sqrt(x.v); return chain(x, s, 0.5 / s); }
inline Dual cbrt(const Dual& x) { double c = std::cbrt(x.v); return chain(x, c, 1.0 / (3.0 * c * c)); }
inline Dual fabs(const Dual& x) { return x.v < 0 ? -x : x; }
inline Dual atan2(const Dual& y, const Dual& x) {
  double den = x.v * x.v + y.v * y.v;
  Dual r(std::atan2(y.v, x.v));
  for (int k = 0; k < kNElem; ++k) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) / den;
  return r;
}
// x - 2*pi*floor(x / 2*pi): the floor is locally constant, so d/dx = 1.
inline Dual mod2pi(const Dual& x) { Dual r = x; r.v = x.v - kTwoPi * std::floor(x.v / kTwoPi); return r; }

// Operation-counting scalar: value in double, every arithmetic operation and
// elementary function call counted once, by kind.
struct OpTally { uint64_t add = 0, mul = 0, div = 0, sqrt = 0, cbrt = 0, trig = 0, atan2 = 0, floor = 0; };
OpTally g_tally;
struct OpCount {
  double v;
  OpCount() : v(0) {}
  OpCount(double x) : v(x) {}  // NOLINT
};
inline double val(const OpCount& x) { return x.v; }
inline OpCount operator+(const OpCount& a, const OpCount& b) { ++g_tally.add; return OpCount(a.v + b.v); }
inline OpCount operator-(const OpCount& a, const OpCount& b) { ++g_tally.add; return OpCount(a.v - b.v); }
inline OpCount operator-(const OpCount& a) { return OpCount(-a.v); }
inline OpCount operator*(const OpCount& a, const OpCount& b) { ++g_tally.mul; return OpCount(a.v * b.v); }
inline OpCount operator/(const OpCount& a, const OpCount& b) { ++g_tally.div; return OpCount(a.v / b.v); }
inline OpCount operator+(const OpCount& a, double b) { return a + OpCount(b); }
inline OpCount operator+(double a, const OpCount& b) { return OpCount(a) + b; }
inline OpCount operator-(const OpCount& a, double b) { return a - OpCount(b); }
inline OpCount operator-(double a, const OpCount& b) { return OpCount(a) - b; }
inline OpCount operator*(const OpCount& a, double b) { return a * OpCount(b); }
inline OpCount operator*(double a, const OpCount& b) { return OpCount(a) * b; }
inline OpCount operator/(const OpCount& a, double b) { return a / OpCount(b); }
inline OpCount operator/(double a, const OpCount& b) { return OpCount(a) / b; }
inline OpCount sin(const OpCount& x) { ++g_tally.trig; return OpCount(std::sin(x.v)); }
inline OpCount cos(const OpCount& x) { ++g_tally.trig; return OpCount(std::cos(x.v)); }
inline OpCount sqrt(const OpCount& x) { ++g_tally.sqrt; return OpCount(std::sqrt(x.v)); }
inline OpCount cbrt(const OpCount& x) { ++g_tally.cbrt; return OpCount(std::cbrt(x.v)); }
inline OpCount fabs(const OpCount& x) { return OpCount(std::fabs(x.v)); }
inline OpCount atan2(const OpCount& y, const OpCount& x) { ++g_tally.atan2; return OpCount(std::atan2(y.v, x.v)); }
inline OpCount mod2pi(const OpCount& x) { ++g_tally.floor; g_tally.mul += 2; ++g_tally.add; return OpCount(x.v - kTwoPi * std::floor(x.v / kTwoPi)); }

inline double mod2pi(double x) { return x - kTwoPi * std::floor(x / kTwoPi); }
using std::atan2;
using std::cbrt;
using std::cos;
using std::fabs;
using std::sin;
using std::sqrt;

template <class S> inline S sq(const S& x) { return x * x; }
template <class S> inline S cube(const S& x) { return x * x * x; }
template <class S> inline S pow4(const S& x) { S x2 = x * x; return x2 * x2; }

// ---------------------------------------------------------------- gravity --
struct Gravity {
  double mu, radius, j2, j3, j4;  // km^3/s^2, km, dimensionless zonals
  double ke;                      // sqrt(mu/R^3) in 1/min: 60/sqrt(R^3/mu)
  double j3oj2;                   // J3/J2, 0 when J3 == 0
  double vkms;                    // earth radii per minute -> km/s: R*ke/60
};

// WGS72 geopotential constants (section 2.1: the paper uses WGS72).
constexpr double kWgs72[5] = {398600.8, 6378.135, 0.001082616, -0.00000253881, -0.00000165597};

int make_gravity(const double* g5, Gravity* g) {
  const double* src = g5 ? g5 : kWgs72;
  g->mu = src[0]; g->radius = src[1]; g->j2 = src[2]; g->j3 = src[3]; g->j4 = src[4];
  if (!(g->mu > 0) || !(g->radius > 0)) return -6;
  if (g->j2 == 0 && g->j3 != 0) return -6;
  g->ke = 60.0 / std::sqrt(g->radius * g->radius * g->radius / g->mu);
  g->j3oj2 = (g->j3 == 0) ? 0.0 : g->j3 / g->j2;
  g->vkms = g->radius * g->ke / 60.0;
  return 0;
}

// --------------------------------------------------------- initialisation --
// Per-satellite constants of the near-Earth model (steps I1-I8).
template <class S>
struct Sat {
  S n0, e0, i0, node0, argp0, M0, bstar;
  double epoch;  // days relative to the caller's reference instant
  S cosi, sini, beta0sq, beta0, c41, x1, x7;
  S n0pp, a0pp, rp, hp, s, q4;
  S xi, eta, C1, C2, C3, C4, C5;
  S Mdot, argpdot, nodedot, nodedot1;
  S argpcof, Mcof, nodecf, t2cof, aycof, Lcof, dM0, sinM0;
  S D2, D3, D4, t3cof, t4cof, t5cof;
  bool isimp = false, deep = false;
  int epoch_code = 0;  // 1 when e0 is outside [0, 1)
  // Deep space (period of 225 min or more): lunar-solar secular rates, the
  // coefficients of the long-period lunar and solar terms (index 0 Sun, 1
  // Moon) and the two bodies' mean anomalies at epoch; resonant orbits are
  // flagged and not propagated.
  bool resonant = false;
  S dedt, didt, dMdt, dnodedt, dargpdt;
  // Resonance (I10): class (1: 24 h, 2: 12 h), the coefficients of its terms
  // (24 h: three; 12 h: ten), the mean longitude of the resonant argument at
  // epoch, its rate apart from the integrated mean motion, and the Greenwich
  // sidereal angle at epoch.
  int irez = 0;
  S res[10];
  S xlamo, xfact;
  double gsto = 0.0;
  S pe2[2], pe3[2], pi2[2], pi3[2], pl2[2], pl3[2], pl4[2], pgh2[2], pgh3[2], pgh4[2], ph2[2], ph3[2];
  double Mbody0[2];
};

// ------------------------------------------------------------ deep space --
// Lunar and solar perturbations of the deep-space model (SDP4: Hujsak 1979,
// in Hoots & Roehrich 1980 as revised by Vallado et al. 2006): the quadrupole
// term of each body's tidal potential, averaged over the satellite's orbit,
// with each body on a fixed-shape orbit whose orientation is set at the
// satellite's epoch.  Secular rates come from the part also averaged over the
// body's mean anomaly; the long-period terms from the rest, to first order in
// the body's eccentricity.  The 12 h and 24 h resonant classes (their
// resonance integrator) are outside this oracle: flagged, not propagated.
//
// The reference instant of the elements' epoch row, as a Julian date (UT):
// the lunar and solar arguments need absolute time.  J2000.0 unless set.
double g_ref_jd = 2451545.0;

// Body constants: mean motion (rad/min), orbital eccentricity, and the
// strength c1 = (mu_body / a_body^3) / (4 n_body), the quadrupole tidal
// coefficient divided by the body's mean motion (the Sun: n_sun / 4; the
// Moon: its mass fraction times n_moon / 4).
constexpr double kNBody[2] = {1.19459e-5, 1.5835218e-4};
constexpr double kEBody[2] = {0.01675, 0.05490};
constexpr double kC1Body[2] = {2.9864797e-6, 4.7968065e-7};
// Obliquity of the ecliptic: sin, cos.  Solar perigee argument: cos, sin.
constexpr double kSinEps = 0.39785416, kCosEps = 0.91744867;
constexpr double kCosSunPer = 0.1945905, kSinSunPer = -0.98088458;
// Moon: sine of its orbit's inclination to the ecliptic; cos of its
// inclination to the equator as kMoonCosI0 - kMoonCosI1 cos(lunar node).
constexpr double kSinMoonInc = 0.089683511;
constexpr double kMoonCosI0 = 0.91375164, kMoonCosI1 = 0.03568096;

// Per-body coefficient set of the averaged quadrupole (the body's orbit given
// by the cos/sin of its perigee argument g, inclination i and the satellite's
// node relative to the body's node h).
template <class S>
struct BodyTerms {
  S s1, s2, s3, s4, s5, s6, s7;
  S z1, z2, z3, z11, z12, z13, z21, z22, z23, z31, z32, z33;
};

template <class S>
BodyTerms<S> body_terms(const S& cg, const S& sg, const S& ci, const S& si, const S& ch, const S& sh,
                        const S& cw, const S& sw, const S& cim, const S& sim, const S& e, double c1,
                        const S& n) {
  BodyTerms<S> b;
  const S e2 = e * e, beta2 = 1.0 - e2, beta = sqrt(beta2);
  // direction cosines of the body's perigee and of the normal-plane axis,
  // first in the satellite's nodal frame (a1..a10), then in its perifocal
  // frame (x1..x8)
  const S a1 = cg * ch + sg * ci * sh;
  const S a3 = -sg * ch + cg * ci * sh;
  const S a7 = -cg * sh + sg * ci * ch;
  const S a8 = sg * si;
  const S a9 = sg * sh + cg * ci * ch;
  const S a10 = cg * si;
  const S a2 = cim * a7 + sim * a8;
  const S a4 = cim * a9 + sim * a10;
  const S a5 = -sim * a7 + cim * a8;
  const S a6 = -sim * a9 + cim * a10;
  const S x1 = a1 * cw + a2 * sw;
  const S x2 = a3 * cw + a4 * sw;
  const S x3 = -a1 * sw + a2 * cw;
  const S x4 = -a3 * sw + a4 * cw;
  const S x5 = a5 * sw;
  const S x6 = a6 * sw;
  const S x7 = a5 * cw;
  const S x8 = a6 * cw;
  b.z31 = 12.0 * x1 * x1 - 3.0 * x3 * x3;
  b.z32 = 24.0 * x1 * x2 - 6.0 * x3 * x4;
  b.z33 = 12.0 * x2 * x2 - 3.0 * x4 * x4;
  const S z1 = 3.0 * (a1 * a1 + a2 * a2) + b.z31 * e2;
  const S z2 = 6.0 * (a1 * a3 + a2 * a4) + b.z32 * e2;
  const S z3 = 3.0 * (a3 * a3 + a4 * a4) + b.z33 * e2;
  b.z11 = -6.0 * a1 * a5 + e2 * (-24.0 * x1 * x7 - 6.0 * x3 * x5);
  b.z12 = -6.0 * (a1 * a6 + a3 * a5) + e2 * (-24.0 * (x2 * x7 + x1 * x8) - 6.0 * (x3 * x6 + x4 * x5));
  b.z13 = -6.0 * a3 * a6 + e2 * (-24.0 * x2 * x8 - 6.0 * x4 * x6);
  b.z21 = 6.0 * a2 * a5 + e2 * (24.0 * x1 * x5 - 6.0 * x3 * x7);
  b.z22 = 6.0 * (a4 * a5 + a2 * a6) + e2 * (24.0 * (x2 * x5 + x1 * x6) - 6.0 * (x4 * x7 + x3 * x8));
  b.z23 = 6.0 * a4 * a6 + e2 * (24.0 * x2 * x6 - 6.0 * x4 * x8);
  b.z1 = 2.0 * z1 + beta2 * b.z31;
  b.z2 = 2.0 * z2 + beta2 * b.z32;
  b.z3 = 2.0 * z3 + beta2 * b.z33;
  b.s3 = c1 / n;
  b.s2 = -0.5 * b.s3 / beta;
  b.s4 = b.s3 * beta;
  b.s1 = -15.0 * e * b.s4;
  b.s5 = x1 * x3 + x2 * x4;
  b.s6 = x2 * x3 + x1 * x4;
  b.s7 = x2 * x4 - x1 * x3;
  return b;
}

// Deep-space initialisation: lunar-solar secular rates, long-period
// coefficients and the bodies' mean anomalies at epoch.  day: days after
// JD 2415020.0 (1900 January 0.5, the origin of the lunar and solar
// arguments).
template <class S>
void deep_init(Sat<S>& c, double day) {
  // The Moon's orbit at epoch: node on the ecliptic, inclination and node on
  // the equator, and its perigee argument from that node.
  const double node_l = mod2pi(4.5236020 - 9.2422029e-4 * day);
  const double sn = std::sin(node_l), cn = std::cos(node_l);
  const double ci_l = kMoonCosI0 - kMoonCosI1 * cn;
  const double si_l = std::sqrt(1.0 - ci_l * ci_l);
  const double sh_l = kSinMoonInc * sn / si_l;
  const double ch_l = std::sqrt(1.0 - sh_l * sh_l);
  const double perigee_l = 5.8351514 + 0.0019443680 * day;
  const double dx = std::atan2(kSinEps * sn / si_l, ch_l * cn + kCosEps * sh_l * sn);
  const double g_l = perigee_l + dx - node_l;
  c.Mbody0[0] = mod2pi(6.2565837 + 0.017201977 * day);
  c.Mbody0[1] = mod2pi(4.7199672 + 0.22997150 * day - perigee_l);

  const S sw = sin(c.argp0), cw = cos(c.argp0);
  const S sni = sin(c.node0), cni = cos(c.node0);
  const S sim = c.sini, cim = c.cosi;
  const S e = c.e0, e2 = e * e;
  BodyTerms<S> b[2];
  // Sun: node of its orbit on the equator at the equinox
  b[0] = body_terms<S>(S(kCosSunPer), S(kSinSunPer), S(kCosEps), S(kSinEps), cni, sni, cw, sw, cim, sim, e,
                       kC1Body[0], c.n0pp);
  // Moon: the satellite's node measured from the Moon's node on the equator
  const S chm = ch_l * cni + sh_l * sni, shm = sni * ch_l - cni * sh_l;
  b[1] = body_terms<S>(S(std::cos(g_l)), S(std::sin(g_l)), S(ci_l), S(si_l), chm, shm, cw, sw, cim, sim, e,
                       kC1Body[1], c.n0pp);
  for (int k = 0; k < 2; ++k) {
    const BodyTerms<S>& q = b[k];
    c.pe2[k] = 2.0 * q.s1 * q.s6;
    c.pe3[k] = 2.0 * q.s1 * q.s7;
    c.pi2[k] = 2.0 * q.s2 * q.z12;
    c.pi3[k] = 2.0 * q.s2 * (q.z13 - q.z11);
    c.pl2[k] = -2.0 * q.s3 * q.z2;
    c.pl3[k] = -2.0 * q.s3 * (q.z3 - q.z1);
    c.pl4[k] = -2.0 * q.s3 * (-21.0 - 9.0 * e2) * kEBody[k];
    c.pgh2[k] = 2.0 * q.s4 * q.z32;
    c.pgh3[k] = 2.0 * q.s4 * (q.z33 - q.z31);
    c.pgh4[k] = -18.0 * q.s4 * kEBody[k];
    c.ph2[k] = -2.0 * q.s2 * q.z22;
    c.ph3[k] = -2.0 * q.s2 * (q.z23 - q.z21);
  }

  // Resonance classes: 24 h (synchronous) and 12 h with e >= 0.5.
  const double nv = val(c.n0pp), ev = val(c.e0);
  c.irez = (nv < 0.0052359877 && nv > 0.0034906585) ? 1 : (nv >= 8.26e-3 && nv <= 9.24e-3 && ev >= 0.5) ? 2 : 0;
  c.resonant = c.irez != 0;

  // Secular rates: the doubly averaged quadrupole in Lagrange's equations.
  // Near-equatorial orbits (inclination within 3 degrees of 0 or 180) take no
  // node rate from the bodies.
  const double iv = val(c.i0);
  const bool flat = iv < 5.2359877e-2 || iv > kPi - 5.2359877e-2;
  S de = S(0.0), di = S(0.0), dM = S(0.0), dgh = S(0.0), dh = S(0.0);
  for (int k = 0; k < 2; ++k) {
    const BodyTerms<S>& q = b[k];
    const double nb = kNBody[k];
    de = de + q.s1 * nb * q.s5;
    di = di + q.s2 * nb * (q.z11 + q.z13);
    dM = dM - nb * q.s3 * (q.z1 + q.z3 - 14.0 - 6.0 * e2);
    dgh = dgh + q.s4 * nb * (q.z31 + q.z33 - 6.0);
    S h = -nb * q.s2 * (q.z21 + q.z23);
    if (flat) h = S(0.0);
    dh = dh + (val(sim) != 0.0 ? h / sim : h);
  }
  c.dedt = de;
  c.didt = di;
  c.dMdt = dM;
  c.dnodedt = dh;
  c.dargpdt = dgh - cim * dh;
}

// ------------------------------------------------------------- resonance --
// Tesseral resonance of the deep-space model (Hoots & Roehrich 1980 as revised
// by Vallado et al. 2006).  An orbit whose mean motion is commensurate with the
// Earth's rotation (24 h: once per sidereal day; 12 h: twice, for e >= 0.5)
// feels tesseral harmonics J_lm of the geopotential secularly, through the
// arguments psi = (l-2p) w + k M + m (node - theta) - m lambda_lm with
// k = l-2p+q.  Lagrange's equation dn/dt = -(3/a^2) dR/dM gives, per term,
// dn/dt = 3 n^2 (R/a)^l k F_lmp(i) G_lpq(e) J_lm sin psi (F: Kaula's
// inclination function, G: the eccentricity function).  Mean motion and the
// mean longitude of the resonant argument (24 h: M + node + w - theta; 12 h:
// M + 2 node - 2 theta) are integrated from epoch with fixed 720-minute
// second-order Taylor steps.

// Earth's rotation rate (rad/min), the integrator's step (min) and its reach
// from epoch (10 Julian years, min): beyond it, or for a time that is not
// finite, the integrated mean motion is NaN (code 2).
constexpr double kEarthRate = 4.37526908801129966e-3;
constexpr double kResStep = 720.0;
constexpr double kResReach = 5259600.0;

// One resonant term: sin(j w + k lambda - phase), with degree l and the
// tesseral magnitude J_lm of the model's geopotential.
struct ResTerm { int j, k, l; double phase, J; };
// 24 h: (l, m) = (3, 1), (2, 2), (3, 3); phases m lambda_lm.
constexpr ResTerm kRes24[3] = {
    {0, 1, 3, 0.13130908, 2.1460748e-6},
    {0, 2, 2, 2.0 * 2.8843198, 1.7891679e-6},
    {0, 3, 3, 3.0 * 0.37448087, 2.2123015e-7}};
// 12 h, in the order (l m p q) = 2201 2211 3210 3222 4410 4422 5220 5232 5421
// 5433 (q signed as k - (l - 2p)).
constexpr ResTerm kRes12[10] = {
    {2, 1, 2, 5.7686396, 1.7891679e-6}, {0, 1, 2, 5.7686396, 1.7891679e-6},
    {1, 1, 3, 0.95240898, 3.7393792e-7}, {-1, 1, 3, 0.95240898, 3.7393792e-7},
    {2, 2, 4, 1.8014998, 7.3636953e-9}, {0, 2, 4, 1.8014998, 7.3636953e-9},
    {1, 1, 5, 1.0508330, 1.1428639e-7}, {-1, 1, 5, 1.0508330, 1.1428639e-7},
    {1, 2, 5, 4.4108898, 2.1765803e-9}, {-1, 2, 5, 4.4108898, 2.1765803e-9}};

// Inclination functions F_lmp(i) of the resonant terms: 24 h (3,1,1),
// (2,2,0), (3,3,0); 12 h (2,2,0), (2,2,1), (3,2,1), (3,2,2), (4,4,1),
// (4,4,2), (5,2,2), (5,2,3), (5,4,2), (5,4,3).
enum { kF311, kF220, kF330, kF221, kF321, kF322, kF441, kF442, kF522, kF523, kF542, kF543, kNF };
template <class S>
void res_inclination(const S& ci, const S& si, S F[kNF]) {
  const S c2 = ci * ci, s2 = si * si;
  F[kF220] = 0.75 * (1.0 + ci) * (1.0 + ci);
  F[kF311] = 0.9375 * s2 * (1.0 + 3.0 * ci) - 0.75 * (1.0 + ci);
  F[kF330] = 1.875 * cube(1.0 + ci);
  F[kF221] = 1.5 * s2;
  F[kF321] = 1.875 * si * (1.0 - 2.0 * ci - 3.0 * c2);
  F[kF322] = -1.875 * si * (1.0 + 2.0 * ci - 3.0 * c2);
  F[kF441] = 35.0 * s2 * F[kF220];
  F[kF442] = 39.375 * s2 * s2;
  F[kF522] = 9.84375 * si * (s2 * (1.0 - 2.0 * ci - 5.0 * c2) + 0.33333333 * (-2.0 + 4.0 * ci + 6.0 * c2));
  F[kF523] = si * (4.92187512 * s2 * (-2.0 - 4.0 * ci + 10.0 * c2) + 6.56250012 * (1.0 + 2.0 * ci - 3.0 * c2));
  F[kF542] = 29.53125 * si * (2.0 - 8.0 * ci + c2 * (-12.0 + 8.0 * ci + 10.0 * c2));
  F[kF543] = 29.53125 * si * (-2.0 - 8.0 * ci + c2 * (12.0 + 8.0 * ci - 10.0 * c2));
}

// Eccentricity functions G_lpq(e): 24 h as series in e (G310, G200, G300);
// 12 h as the model's polynomial fits over e >= 0.5 (G201, G211, G310, G322,
// G410, G422, G520, G532, G521, G533; q = -1 for G201).
enum { kG310s, kG200, kG300, kG201, kG211, kG310, kG322, kG410, kG422, kG520, kG532, kG521, kG533, kNG };
template <class S>
void res_eccentricity(const S& e, S G[kNG]) {
  const S e2 = e * e, e3 = e2 * e;
  G[kG310s] = 1.0 + 2.0 * e2;
  G[kG200] = 1.0 + e2 * (-2.5 + 0.8125 * e2);
  G[kG300] = 1.0 + e2 * (-6.0 + 6.60937 * e2);
  G[kG201] = -0.306 - (e - 0.64) * 0.440;
  if (val(e) <= 0.65) {
    G[kG211] = 3.616 - 13.2470 * e + 16.2900 * e2;
    G[kG310] = -19.302 + 117.3900 * e - 228.4190 * e2 + 156.5910 * e3;
    G[kG322] = -18.9068 + 109.7927 * e - 214.6334 * e2 + 146.5816 * e3;
    G[kG410] = -41.122 + 242.6940 * e - 471.0940 * e2 + 313.9530 * e3;
    G[kG422] = -146.407 + 841.8800 * e - 1629.014 * e2 + 1083.4350 * e3;
    G[kG520] = -532.114 + 3017.977 * e - 5740.032 * e2 + 3708.2760 * e3;
  } else {
    G[kG211] = -72.099 + 331.819 * e - 508.738 * e2 + 266.724 * e3;
    G[kG310] = -346.844 + 1582.851 * e - 2415.925 * e2 + 1246.113 * e3;
    G[kG322] = -342.585 + 1554.908 * e - 2366.899 * e2 + 1215.972 * e3;
    G[kG410] = -1052.797 + 4758.686 * e - 7193.992 * e2 + 3651.957 * e3;
    G[kG422] = -3581.690 + 16178.110 * e - 24462.770 * e2 + 12422.520 * e3;
    if (val(e) > 0.715)
      G[kG520] = -5149.66 + 29936.92 * e - 54087.36 * e2 + 31324.56 * e3;
    else
      G[kG520] = 1464.74 - 4664.75 * e + 3763.64 * e2;
  }
  if (val(e) < 0.7) {
    G[kG533] = -919.22770 + 4988.6100 * e - 9064.7700 * e2 + 5542.21 * e3;
    G[kG521] = -822.71072 + 4568.6173 * e - 8491.4146 * e2 + 5337.524 * e3;
    G[kG532] = -853.66600 + 4690.2500 * e - 8624.7700 * e2 + 5341.4 * e3;
  } else {
    G[kG533] = -37995.780 + 161616.52 * e - 229838.20 * e2 + 109377.94 * e3;
    G[kG521] = -51752.104 + 218913.95 * e - 309468.16 * e2 + 146349.42 * e3;
    G[kG532] = -40023.880 + 170470.89 * e - 242699.48 * e2 + 115605.82 * e3;
  }
}

// IAU 1982 Greenwich mean sidereal time (Aoki et al. 1982) at a Julian date
// taken as UT1, radians in [0, 2 pi): seconds of sidereal time as a cubic in
// Julian centuries from J2000.0, the 12 h offset of that epoch included.
double gmst_iau82(double day1900) {
  const double T = (day1900 - 36525.0) / 36525.0;  // J2000.0 is day 36525 after JD 2415020.0
  const double sec = 67310.54841 + (876600.0 * 3600.0 + 8640184.812866) * T + 0.093104 * T * T - 6.2e-6 * T * T * T;
  double x = std::fmod(sec, 86400.0) * (kTwoPi / 86400.0);
  if (x < 0.0) x += kTwoPi;
  return x;
}

// One term's coefficient 3 n^2 (R/a)^l k J F G, from base = 3 n^2 (R/a)^2.
template <class S>
S res_coef(const S& base, const S& ra, const ResTerm& q, const S& FG) {
  S coef = base * double(q.k) * q.J * FG;
  for (int l = 2; l < q.l; ++l) coef = coef * ra;
  return coef;
}

// I10 (resonant deep space): term coefficients 3 n^2 (R/a)^l k J F G, the
// resonant mean longitude at epoch and its rate apart from the mean motion:
// the secular rates of M, w and node (gravity and the bodies) minus the
// Earth's rotation, taken m times.
template <class S>
void resonance_init(const Gravity& g, Sat<S>& c, double day) {
  c.gsto = gmst_iau82(day);
  if (!c.irez) return;
  const S ra = sq(cbrt(c.n0pp / g.ke));  // R/a
  const S base = 3.0 * c.n0pp * c.n0pp * ra * ra;
  S F[kNF], G[kNG];
  res_inclination(c.cosi, c.sini, F);
  res_eccentricity(c.e0, G);
  if (c.irez == 1) {
    const S FG[3] = {F[kF311] * G[kG310s], F[kF220] * G[kG200], F[kF330] * G[kG300]};
    for (int k = 0; k < 3; ++k) c.res[k] = res_coef(base, ra, kRes24[k], FG[k]);
    c.xlamo = mod2pi(c.M0 + c.node0 + c.argp0 - c.gsto);
    c.xfact = c.Mdot + (c.argpdot + c.nodedot) - kEarthRate + c.dMdt + c.dargpdt + c.dnodedt - c.n0pp;
  } else {
    const S FG[10] = {F[kF220] * G[kG201], F[kF221] * G[kG211], F[kF321] * G[kG310], F[kF322] * G[kG322],
                      F[kF441] * G[kG410], F[kF442] * G[kG422], F[kF522] * G[kG520], F[kF523] * G[kG532],
                      F[kF542] * G[kG521], F[kF543] * G[kG533]};
    for (int k = 0; k < 10; ++k) c.res[k] = res_coef(base, ra, kRes12[k], FG[k]);
    c.xlamo = mod2pi(c.M0 + 2.0 * c.node0 - 2.0 * c.gsto);
    c.xfact = c.Mdot + c.dMdt + 2.0 * (c.nodedot + c.dnodedt - kEarthRate) - c.n0pp;
  }
}

// Resonance rates at mean longitude xli and mean motion xni, atime minutes
// after epoch (the perigee argument of the 12 h terms advanced by its
// gravity rate): dn/dt, its time derivative along the resonant argument, and
// d(lambda)/dt.
template <class S>
void res_rates(const Sat<S>& c, const S& xli, const S& xni, double atime, S* ndot, S* nddot, S* ldot) {
  const int nt = c.irez == 1 ? 3 : 10;
  const ResTerm* terms = c.irez == 1 ? kRes24 : kRes12;
  const S w = c.argp0 + c.argpdot * atime;
  S sn = S(0.0), cs = S(0.0);
  for (int k = 0; k < nt; ++k) {
    const ResTerm& q = terms[k];
    const S arg = double(q.j) * w + double(q.k) * xli - q.phase;
    sn = sn + c.res[k] * sin(arg);
    cs = cs + double(q.k) * c.res[k] * cos(arg);
  }
  *ldot = xni + c.xfact;
  *ndot = sn;
  *nddot = cs * *ldot;
}

// P3r: integrate (lambda, n) from epoch to t in steps of 720 minutes toward t
// while at least a whole step remains, then the Taylor polynomial over the
// remainder.  Returns the time of the last step.
template <class S>
double res_integrate(const Sat<S>& c, double t, S* xl, S* nm) {
  S xli = c.xlamo, xni = c.n0pp, ndot, nddot, ldot;
  double atime = 0.0;
  const double h = t > 0.0 ? kResStep : -kResStep;
  if (!(std::fabs(t) <= kResReach)) {
    *xl = *nm = S(std::numeric_limits<double>::quiet_NaN());
    return 0.0;
  }
  for (;;) {
    res_rates(c, xli, xni, atime, &ndot, &nddot, &ldot);
    if (!(std::fabs(t - atime) >= kResStep)) break;
    xli = xli + ldot * h + ndot * (0.5 * h * h);
    xni = xni + ndot * h + nddot * (0.5 * h * h);
    atime += h;
  }
  const double ft = t - atime;
  *nm = xni + ndot * ft + nddot * (0.5 * ft * ft);
  *xl = xli + ldot * ft + ndot * (0.5 * ft * ft);
  return atime;
}

template <class S>
Sat<S> sgp4_init(const Gravity& g, const S el[kNElem], double epoch) {
  Sat<S> c;
  c.n0 = el[0]; c.e0 = el[1]; c.i0 = el[2]; c.node0 = el[3]; c.argp0 = el[4]; c.M0 = el[5]; c.bstar = el[6];
  c.epoch = epoch;
  const double R = g.radius, J2 = g.j2, J4 = g.j4, ke = g.ke, j3oj2 = g.j3oj2;
  const S& n0 = c.n0; const S& e0 = c.e0;
  if (!(val(e0) >= 0.0 && val(e0) < 1.0)) c.epoch_code = 1;

  // I1: inclination and eccentricity functions.
  c.cosi = cos(c.i0);
  c.sini = sin(c.i0);
  S th2 = c.cosi * c.cosi;
  c.beta0sq = 1.0 - e0 * e0;
  c.beta0 = sqrt(c.beta0sq);
  c.c41 = 3.0 * th2 - 1.0;
  c.x1 = 1.0 - th2;
  c.x7 = 7.0 * th2 - 1.0;

  // I2: recover the original (Brouwer) mean motion and semi-major axis from
  // the Kozai mean motion of the element set.
  S a1 = sq(cbrt(ke / n0));
  S d1 = 0.75 * J2 * c.c41 / (c.beta0 * c.beta0sq);
  S del1 = d1 / (a1 * a1);
  S adel = a1 * (1.0 - del1 / 3.0 - del1 * del1 - (134.0 / 81.0) * del1 * del1 * del1);
  S del0 = d1 / (adel * adel);
  c.n0pp = n0 / (1.0 + del0);
  c.a0pp = sq(cbrt(ke / c.n0pp));

  // I3: perigee height selects the atmospheric density parameter s and q0-s.
  c.rp = c.a0pp * (1.0 - e0);
  c.hp = (c.rp - 1.0) * R;
  c.s = S(1.0 + 78.0 / R);
  c.q4 = S(pow4((120.0 - 78.0) / R));
  if (val(c.hp) < 156.0) {
    S sstar = c.hp - 78.0;
    if (val(c.hp) < 98.0) sstar = S(20.0);
    c.q4 = pow4((120.0 - sstar) / R);
    c.s = 1.0 + sstar / R;
  }

  // I4: flags.  Deep space: period 2*pi/n0'' of 225 min or more.  Simplified
  // drag: perigee below 220 km.
  c.deep = (val(c.n0pp) > 0.0) && (kTwoPi / val(c.n0pp) >= 225.0);
  c.isimp = c.deep || val(c.rp) < 1.0 + 220.0 / R;

  // I5: drag coefficients.
  c.xi = 1.0 / (c.a0pp - c.s);
  c.eta = c.a0pp * e0 * c.xi;
  S eta2 = c.eta * c.eta;
  S e0eta = e0 * c.eta;
  S q = fabs(1.0 - eta2);
  S coef = c.q4 * pow4(c.xi);
  S coef1 = coef / (q * q * q * sqrt(q));
  c.C2 = coef1 * c.n0pp *
         (c.a0pp * (1.0 + 1.5 * eta2 + e0eta * (4.0 + eta2)) +
          0.375 * J2 * c.xi / q * c.c41 * (8.0 + 3.0 * eta2 * (8.0 + eta2)));
  c.C1 = c.bstar * c.C2;
  c.C3 = S(0.0);
  if (val(e0) > 1.0e-4) c.C3 = -2.0 * coef * c.xi * j3oj2 * c.n0pp * c.sini / e0;
  c.C4 = 2.0 * c.n0pp * coef1 * c.a0pp * c.beta0sq *
         (c.eta * (2.0 + 0.5 * eta2) + e0 * (0.5 + 2.0 * eta2) -
          J2 * c.xi / (c.a0pp * q) *
              (-3.0 * c.c41 * (1.0 - 2.0 * e0eta + eta2 * (1.5 - 0.5 * e0eta)) +
               0.75 * c.x1 * (2.0 * eta2 - e0eta * (1.0 + eta2)) * cos(2.0 * c.argp0)));
  c.C5 = 2.0 * coef1 * c.a0pp * c.beta0sq * (1.0 + 2.75 * (eta2 + e0eta) + e0eta * eta2);

  // I6: secular rates of M, argument of perigee and node (J2, J2^2, J4).
  S p0 = c.a0pp * c.beta0sq;
  S p0sq = p0 * p0;
  S T1 = 1.5 * J2 * c.n0pp / p0sq;
  S T2 = 0.5 * T1 * J2 / p0sq;
  S T3 = -(15.0 / 32.0) * J4 * c.n0pp / (p0sq * p0sq);
  S th4 = th2 * th2;
  c.Mdot = c.n0pp + 0.5 * T1 * c.beta0 * c.c41 + (1.0 / 16.0) * T2 * c.beta0 * (13.0 - 78.0 * th2 + 137.0 * th4);
  c.argpdot = -0.5 * T1 * (1.0 - 5.0 * th2) + (1.0 / 16.0) * T2 * (7.0 - 114.0 * th2 + 395.0 * th4) +
              T3 * (3.0 - 36.0 * th2 + 49.0 * th4);
  c.nodedot1 = -T1 * c.cosi;
  c.nodedot = c.nodedot1 + (0.5 * T2 * (4.0 - 19.0 * th2) + 2.0 * T3 * (3.0 - 7.0 * th2)) * c.cosi;

  // I7: drag-on-angles and long-period (J3) coefficients.
  c.argpcof = c.bstar * c.C3 * cos(c.argp0);
  c.Mcof = S(0.0);
  if (val(e0) > 1.0e-4) c.Mcof = -(2.0 / 3.0) * coef * c.bstar / e0eta;
  c.nodecf = 3.5 * c.beta0sq * c.nodedot1 * c.C1;
  c.t2cof = 1.5 * c.C1;
  c.aycof = -0.5 * j3oj2 * c.sini;
  S den = 1.0 + c.cosi;
  if (std::fabs(val(den)) <= 1.5e-12) den = S(1.5e-12);
  c.Lcof = -0.25 * j3oj2 * c.sini * (3.0 + 5.0 * c.cosi) / den;
  c.dM0 = cube(1.0 + c.eta * cos(c.M0));
  c.sinM0 = sin(c.M0);

  // I8: higher-order drag terms (only when the simplified model is off).
  c.D2 = c.D3 = c.D4 = c.t3cof = c.t4cof = c.t5cof = S(0.0);
  if (!c.isimp) {
    S C1sq = c.C1 * c.C1;
    c.D2 = 4.0 * c.a0pp * c.xi * C1sq;
    c.D3 = (4.0 / 3.0) * c.a0pp * c.xi * c.xi * (17.0 * c.a0pp + c.s) * C1sq * c.C1;
    c.D4 = (2.0 / 3.0) * c.a0pp * c.a0pp * c.xi * c.xi * c.xi * (221.0 * c.a0pp + 31.0 * c.s) * C1sq * C1sq;
    c.t3cof = c.D2 + 2.0 * C1sq;
    c.t4cof = 0.25 * (3.0 * c.D3 + c.C1 * (12.0 * c.D2 + 10.0 * C1sq));
    c.t5cof = 0.2 * (3.0 * c.D4 + 12.0 * c.C1 * c.D3 + 6.0 * c.D2 * c.D2 + 15.0 * C1sq * (2.0 * c.D2 + C1sq));
  }
  c.dedt = c.didt = c.dMdt = c.dnodedt = c.dargpdt = S(0.0);
  c.Mbody0[0] = c.Mbody0[1] = 0.0;
  for (int k = 0; k < 2; ++k)
    c.pe2[k] = c.pe3[k] = c.pi2[k] = c.pi3[k] = c.pl2[k] = c.pl3[k] = c.pl4[k] = c.pgh2[k] = c.pgh3[k] =
        c.pgh4[k] = c.ph2[k] = c.ph3[k] = S(0.0);
  // I9: deep space.  The epoch in days after 1900 January 0.5.
  // I10: resonance (after the secular rates it adds to).
  c.irez = 0;
  c.xlamo = c.xfact = S(0.0);
  for (int k = 0; k < 10; ++k) c.res[k] = S(0.0);
  if (c.deep && !c.epoch_code) {
    const double day = (g_ref_jd - 2415020.0) + epoch;
    deep_init(c, day);
    resonance_init(g, c, day);
  }
  return c;
}

// Long-period lunar-solar terms at time t after epoch (each body's mean
// anomaly advanced by its mean motion, its true anomaly to first order in
// its eccentricity): the changes of e, i, M, argp + node and node.
template <class S>
void deep_periodics(const Sat<S>& c, double t, S* pe, S* pinc, S* pl, S* pgh, S* ph) {
  *pe = *pinc = *pl = *pgh = *ph = S(0.0);
  for (int k = 0; k < 2; ++k) {
    const double Mb = c.Mbody0[k] + kNBody[k] * t;
    const double f = Mb + 2.0 * kEBody[k] * std::sin(Mb);
    const double sf = std::sin(f);
    const double f2 = 0.5 * sf * sf - 0.25;
    const double f3 = -0.5 * sf * std::cos(f);
    *pe = *pe + c.pe2[k] * f2 + c.pe3[k] * f3;
    *pinc = *pinc + c.pi2[k] * f2 + c.pi3[k] * f3;
    *pl = *pl + c.pl2[k] * f2 + c.pl3[k] * f3 + c.pl4[k] * sf;
    *pgh = *pgh + c.pgh2[k] * f2 + c.pgh3[k] * f3 + c.pgh4[k] * sf;
    *ph = *ph + c.ph2[k] * f2 + c.ph3[k] * f3;
  }
}

// ------------------------------------------------------------ propagation --
// Intermediate values of one point, exposed for the structural pins.
enum DetailIdx {
  kD_M, kD_argp, kD_node, kD_a, kD_n, kD_e, kD_L, kD_axn, kD_ayn, kD_LT, kD_U, kD_psi, kD_iters, kD_resid,
  kD_ecE, kD_esE, kD_eL2, kD_pL, kD_r, kD_rdot, kD_rfdot, kD_betaL, kD_sinu, kD_cosu, kD_u,
  kD_k1, kD_k2, kD_rk, kD_uk, kD_nodek, kD_ik, kD_rdotk, kD_rfdotk, kD_code, kD_emargin, kD_COUNT
};

inline double wrap_pi(double x) { return x - kTwoPi * std::floor((x + kPi) / kTwoPi); }

template <class S>
int sgp4_point(const Gravity& g, const Sat<S>& c, double tsince, S r[3], S v[3], double* det) {
  const double nan = std::numeric_limits<double>::quiet_NaN();
  auto fail = [&](int code) {
    for (int k = 0; k < 3; ++k) { r[k] = S(nan); v[k] = S(nan); }
    if (det) det[kD_code] = code;
    return code;
  };
  if (det) for (int k = 0; k < kD_COUNT; ++k) det[k] = nan;
  if (c.epoch_code) return fail(1);
  if (!(val(c.n0pp) > 0.0)) return fail(2);

  const double t = tsince;
  const double t2 = t * t;
  // P1: secular gravity.
  S M_df = c.M0 + c.Mdot * t;
  S argp_df = c.argp0 + c.argpdot * t;
  S node_df = c.node0 + c.nodedot * t;
  S node = node_df + c.nodecf * t2;
  // P2: secular drag.
  S A = 1.0 - c.C1 * t;
  S Ed = c.bstar * c.C4 * t;
  S Ld = c.t2cof * t2;
  S M, argp;
  if (!c.isimp) {
    S dargp = c.argpcof * t;
    S dM = c.Mcof * (cube(1.0 + c.eta * cos(M_df)) - c.dM0);
    M = M_df + dargp + dM;
    argp = argp_df - dargp - dM;
    const double t3 = t2 * t, t4 = t3 * t;
    A = A - c.D2 * t2 - c.D3 * t3 - c.D4 * t4;
    Ed = Ed + c.bstar * c.C5 * (sin(M) - c.sinM0);
    Ld = Ld + c.t3cof * t3 + t4 * (c.t4cof + t * c.t5cof);
  } else {
    M = M_df;
    argp = argp_df;
  }
  // P2d (deep space): lunar-solar secular rates.
  S e_sec = c.e0, incl = c.i0;
  if (c.deep) {
    e_sec = e_sec + c.dedt * t;
    incl = incl + c.didt * t;
    argp = argp + c.dargpdt * t;
    node = node + c.dnodedt * t;
    M = M + c.dMdt * t;
  }
  // P3r (resonant deep space): the mean anomaly from the integrated resonant
  // longitude and the Greenwich sidereal angle at t; the semi-major axis from
  // the integrated mean motion.
  S a0 = c.a0pp;
  if (c.irez) {
    S xl, nm;
    res_integrate(c, t, &xl, &nm);
    const double theta = mod2pi(c.gsto + t * kEarthRate);
    if (c.irez == 1)
      M = xl - node - argp + theta;
    else
      M = xl - 2.0 * node + 2.0 * theta;
    if (!(val(nm) > 0.0)) return fail(2);
    a0 = sq(cbrt(g.ke / nm));
  }
  // P3: drag-decayed semi-major axis, mean motion and eccentricity.
  S a = a0 * A * A;
  S n = g.ke / (a * sqrt(a));
  S e = e_sec - Ed;
  if (det) det[kD_emargin] = std::min(val(e) + 0.001, 1.0 - val(e));
  if (!(val(e) >= -0.001 && val(e) < 1.0)) return fail(1);
  if (val(e) < 1.0e-6) e = S(1.0e-6);
  // P4: mean longitude; angles reduced to [0, 2*pi).
  M = M + c.n0pp * Ld;
  S L = M + argp + node;
  node = mod2pi(node);
  argp = mod2pi(argp);
  L = mod2pi(L);
  // Inclination functions of the periodic terms: the epoch's, except in deep
  // space, where the lunar-solar terms move the inclination.
  S incp = c.i0, sinip = c.sini, cosip = c.cosi, c41 = c.c41, x1 = c.x1, x7 = c.x7;
  S aycof = c.aycof, Lcof = c.Lcof;
  S LT, U, axn, ayn, tau;
  if (!c.deep) {
    // P5: long-period periodics (J3).
    axn = e * cos(argp);
    tau = 1.0 / (a * (1.0 - e * e));
    ayn = e * sin(argp) + tau * aycof;
    LT = L + tau * Lcof * axn;
    U = mod2pi(LT - node);
  } else {
    // P4d: long-period lunar-solar terms on the mean elements.
    M = mod2pi(L - argp - node);
    S pe, pinc, pl, pgh, ph;
    deep_periodics(c, t, &pe, &pinc, &pl, &pgh, &ph);
    incp = incl + pinc;
    e = e + pe;
    sinip = sin(incp);
    cosip = cos(incp);
    if (val(incp) >= 0.2) {
      ph = ph / sinip;
      pgh = pgh - cosip * ph;
      argp = argp + pgh;
      node = node + ph;
      M = M + pl;
    } else {
      // Low inclination: the node and inclination changes applied to the
      // components (sin i sin node, sin i cos node), and the longitude
      // argp + cos i node carried through, so that nothing divides by sin i.
      S sno = sin(node), cno = cos(node);
      S alf = sinip * sno + (ph * cno + pinc * cosip * sno);
      S bet = sinip * cno + (-ph * sno + pinc * cosip * cno);
      node = mod2pi(node);
      S xls = M + argp + cosip * node + (pl + pgh - pinc * node * sinip);
      S node_old = node;
      node = atan2(alf, bet);
      if (std::fabs(val(node_old) - val(node)) > kPi) node = val(node) < val(node_old) ? node + kTwoPi : node - kTwoPi;
      M = M + pl;
      argp = xls - M - cosip * node;
    }
    if (val(incp) < 0.0) {
      incp = -incp;
      node = node + kPi;
      argp = argp - kPi;
    }
    if (det) det[kD_e] = val(e);
    if (!(val(e) >= 0.0 && val(e) <= 1.0)) return fail(3);
    sinip = sin(incp);
    cosip = cos(incp);
    const S cos2 = cosip * cosip;
    c41 = 3.0 * cos2 - 1.0;
    x1 = 1.0 - cos2;
    x7 = 7.0 * cos2 - 1.0;
    aycof = -0.5 * g.j3oj2 * sinip;
    S den = 1.0 + cosip;
    if (std::fabs(val(den)) <= 1.5e-12) den = S(1.5e-12);
    Lcof = -0.25 * g.j3oj2 * sinip * (3.0 + 5.0 * cosip) / den;
    // P5: long-period periodics (J3) with the perturbed elements.
    axn = e * cos(argp);
    tau = 1.0 / (a * (1.0 - e * e));
    ayn = e * sin(argp) + tau * aycof;
    LT = M + argp + node + tau * Lcof * axn;
    U = mod2pi(LT - node);
  }
  // P6: Kepler's equation for psi = E + argp:  psi - axn sin psi + ayn cos psi = U.
  S psi = U;
  int iters = 0;
  for (int k = 0; k < 10; ++k) {
    S sp = sin(psi), cp = cos(psi);
    S step = (U - ayn * cp + axn * sp - psi) / (1.0 - axn * cp - ayn * sp);
    if (val(step) > 0.95) step = S(0.95);
    if (val(step) < -0.95) step = S(-0.95);
    psi = psi + step;
    ++iters;
    if (std::fabs(val(step)) < 1.0e-12) break;
  }
  S sinpsi = sin(psi), cospsi = cos(psi);
  // P7: short-period preliminaries.
  S ecE = axn * cospsi + ayn * sinpsi;
  S esE = axn * sinpsi - ayn * cospsi;
  S eL2 = axn * axn + ayn * ayn;
  S pL = a * (1.0 - eL2);
  if (det) {
    det[kD_M] = val(M); det[kD_argp] = val(argp); det[kD_node] = val(node); det[kD_a] = val(a);
    det[kD_n] = val(n); det[kD_e] = val(e); det[kD_L] = val(L); det[kD_axn] = val(axn); det[kD_ayn] = val(ayn);
    det[kD_LT] = val(LT); det[kD_U] = val(U); det[kD_psi] = val(psi); det[kD_iters] = iters;
    det[kD_resid] = wrap_pi(val(psi) - val(axn) * std::sin(val(psi)) + val(ayn) * std::cos(val(psi)) - val(U));
    det[kD_ecE] = val(ecE); det[kD_esE] = val(esE); det[kD_eL2] = val(eL2); det[kD_pL] = val(pL);
  }
  if (!(val(pL) >= 0.0)) return fail(4);
  S rr = a * (1.0 - ecE);
  S rdot = sqrt(a) * esE / rr;
  S rfdot = sqrt(pL) / rr;
  S betaL = sqrt(1.0 - eL2);
  S w = esE / (1.0 + betaL);
  S sinu = a / rr * (sinpsi - ayn - axn * w);
  S cosu = a / rr * (cospsi - axn + ayn * w);
  S u = atan2(sinu, cosu);
  S sin2u = 2.0 * sinu * cosu;
  S cos2u = 1.0 - 2.0 * sinu * sinu;
  // P8: short-period periodics (J2).
  S k1 = 0.5 * g.j2 / pL;
  S k2 = k1 / pL;
  S rk = rr * (1.0 - 1.5 * k2 * betaL * c41) + 0.5 * k1 * x1 * cos2u;
  S uk = u - 0.25 * k2 * x7 * sin2u;
  S nodek = node + 1.5 * k2 * cosip * sin2u;
  S ik = incp + 1.5 * k2 * cosip * sinip * cos2u;
  S rdotk = rdot - n / g.ke * k1 * x1 * sin2u;
  S rfdotk = rfdot + n / g.ke * k1 * (x1 * cos2u + 1.5 * c41);
  // P9: orientation vectors and the TEME state.
  S su = sin(uk), cu = cos(uk), sn = sin(nodek), cn = cos(nodek), si = sin(ik), ci = cos(ik);
  S mx = -sn * ci, my = cn * ci, mz = si;
  S ux = mx * su + cn * cu, uy = my * su + sn * cu, uz = mz * su;
  S vx = mx * cu - cn * su, vy = my * cu - sn * su, vz = mz * cu;
  r[0] = g.radius * rk * ux; r[1] = g.radius * rk * uy; r[2] = g.radius * rk * uz;
  v[0] = g.vkms * (rdotk * ux + rfdotk * vx);
  v[1] = g.vkms * (rdotk * uy + rfdotk * vy);
  v[2] = g.vkms * (rdotk * uz + rfdotk * vz);
  int code = (val(rk) < 1.0) ? 6 : 0;
  if (det) {
    det[kD_r] = val(rr); det[kD_rdot] = val(rdot); det[kD_rfdot] = val(rfdot); det[kD_betaL] = val(betaL);
    det[kD_sinu] = val(sinu); det[kD_cosu] = val(cosu); det[kD_u] = val(u); det[kD_k1] = val(k1); det[kD_k2] = val(k2);
    det[kD_rk] = val(rk); det[kD_uk] = val(uk); det[kD_nodek] = val(nodek); det[kD_ik] = val(ik);
    det[kD_rdotk] = val(rdotk); det[kD_rfdotk] = val(rfdotk); det[kD_code] = code;
  }
  return code;
}

// ------------------------------------------------------------ batch glue --
template <class F>
void parallel_for(int64_t n, int nthreads, F&& body) {
  if (nthreads <= 1 || n < 2) { body(int64_t(0), n); return; }
  nthreads = int(std::min<int64_t>(nthreads, n));
  std::vector<std::thread> pool;
  for (int k = 0; k < nthreads; ++k) {
    int64_t lo = n * k / nthreads, hi = n * (k + 1) / nthreads;
    pool.emplace_back([&body, lo, hi] { body(lo, hi); });
  }
  for (auto& th : pool) th.join();
}

template <class S>
void load_elements(const double* elem, int64_t n, int64_t i, S el[kNElem], double* epoch) {
  for (int k = 0; k < kNElem; ++k) el[k] = S(elem[k * n + i]);
  *epoch = elem[7 * n + i];
}

void store_point(const double r[3], const double v[3], int code, int64_t P, int64_t p, double* ro, double* vo, uint8_t* err) {
  for (int k = 0; k < 3; ++k) { ro[k * P + p] = r[k]; vo[k * P + p] = v[k]; }
  err[p] = uint8_t(code);
}

}  // namespace

// ================================================================== C ABI ==
// Layouts: elem is [8][n] row-major (rows: no_kozai rad/min, ecco, inclo rad,
// nodeo rad, argpo rad, mo rad, bstar 1/earth-radii, epoch days relative to
// the caller's reference).  Times are minutes after that reference; the time
// since epoch is t - 1440*epoch.  r, v are [3][P] in km and km/s; err is [P].
// grav is NULL (WGS72) or {mu, R, J2, J3, J4}.  Returns 0 or a negative code.
extern "C" {

int oracle_abi_version(void) { return 1; }

// Reference instant of the elements' epoch row and of the times, as a Julian
// date (whole + fraction); used only by the deep-space model's lunar and
// solar arguments.  J2000.0 by default.
void oracle_set_reference_jd(double whole, double frac) { g_ref_jd = whole + frac; }
double oracle_reference_jd(void) { return g_ref_jd; }

void oracle_wgs72(double* out5) { for (int k = 0; k < 5; ++k) out5[k] = kWgs72[k]; }

double oracle_ke(const double* grav) { Gravity g; if (make_gravity(grav, &g)) return -1; return g.ke; }

int oracle_propagate(const double* grav, int64_t n, const double* elem, const double* t, int64_t T,
                     double* r, double* v, uint8_t* err, int nthreads) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  if (n < 0 || T < 0) return -2;
  const int64_t P = n * T;
  parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      double el[kNElem], epoch;
      load_elements(elem, n, i, el, &epoch);
      Sat<double> c = sgp4_init<double>(g, el, epoch);
      for (int64_t j = 0; j < T; ++j) {
        double rr[3], vv[3];
        int code = sgp4_point(g, c, t[j] - 1440.0 * epoch, rr, vv, nullptr);
        store_point(rr, vv, code, P, i * T + j, r, v, err);
      }
    }
  });
  return 0;
}

int oracle_propagate_ragged(const double* grav, int64_t n, const double* elem, const int64_t* offsets,
                            const double* t, int64_t nnz, double* r, double* v, uint8_t* err, int nthreads) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  if (n < 0 || nnz < 0 || offsets[0] != 0 || offsets[n] != nnz) return -3;
  for (int64_t i = 0; i < n; ++i) if (offsets[i + 1] < offsets[i]) return -3;
  parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      double el[kNElem], epoch;
      load_elements(elem, n, i, el, &epoch);
      Sat<double> c = sgp4_init<double>(g, el, epoch);
      for (int64_t p = offsets[i]; p < offsets[i + 1]; ++p) {
        double rr[3], vv[3];
        int code = sgp4_point(g, c, t[p] - 1440.0 * epoch, rr, vv, nullptr);
        store_point(rr, vv, code, nnz, p, r, v, err);
      }
    }
  });
  return 0;
}

// Codes only, over CSR lists (the same definition as oracle_propagate_ragged;
// the states are computed and dropped), for code checks of batches whose
// states would not fit in host memory.
int oracle_codes_ragged(const double* grav, int64_t n, const double* elem, const int64_t* offsets,
                        const double* t, int64_t nnz, uint8_t* err, int nthreads) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  if (n < 0 || nnz < 0 || offsets[0] != 0 || offsets[n] != nnz) return -3;
  for (int64_t i = 0; i < n; ++i) if (offsets[i + 1] < offsets[i]) return -3;
  parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      double el[kNElem], epoch;
      load_elements(elem, n, i, el, &epoch);
      Sat<double> c = sgp4_init<double>(g, el, epoch);
      for (int64_t p = offsets[i]; p < offsets[i + 1]; ++p) {
        double rr[3], vv[3];
        err[p] = uint8_t(sgp4_point(g, c, t[p] - 1440.0 * epoch, rr, vv, nullptr));
      }
    }
  });
  return 0;
}

// Individual (satellite, time) points: sat[k] indexes the n element sets, t[k]
// is minutes after the reference.  Optional detail[k][kD_COUNT] intermediates.
int oracle_propagate_points(const double* grav, int64_t n, const double* elem, int64_t npts, const int64_t* sat,
                            const double* t, double* r, double* v, uint8_t* err, double* detail) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  for (int64_t k = 0; k < npts; ++k) {
    if (sat[k] < 0 || sat[k] >= n) return -1;
    double el[kNElem], epoch;
    load_elements(elem, n, sat[k], el, &epoch);
    Sat<double> c = sgp4_init<double>(g, el, epoch);
    double rr[3], vv[3];
    int code = sgp4_point(g, c, t[k] - 1440.0 * epoch, rr, vv, detail ? detail + k * kD_COUNT : nullptr);
    store_point(rr, vv, code, npts, k, r, v, err);
  }
  return 0;
}

int oracle_detail_count(void) { return kD_COUNT; }

// Initialisation constants per satellite, [n][kI_COUNT] in this order.
enum { kI_COUNT = 90 };
int oracle_init_count(void) { return kI_COUNT; }
int oracle_init(const double* grav, int64_t n, const double* elem, double* rec) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  for (int64_t i = 0; i < n; ++i) {
    double el[kNElem], epoch;
    load_elements(elem, n, i, el, &epoch);
    Sat<double> c = sgp4_init<double>(g, el, epoch);
    double out[kI_COUNT] = {
        c.cosi, c.sini, c.beta0sq, c.beta0, c.c41, c.x1, c.x7, c.n0pp, c.a0pp, c.rp, c.hp, c.s, c.q4,
        c.xi, c.eta, c.C1, c.C2, c.C3, c.C4, c.C5, c.Mdot, c.argpdot, c.nodedot, c.nodedot1,
        c.argpcof, c.Mcof, c.nodecf, c.t2cof, c.aycof, c.Lcof, c.dM0, c.sinM0,
        c.D2, c.D3, c.D4, c.t3cof, c.t4cof, c.t5cof, double(c.isimp), double(c.deep), double(c.epoch_code),
        g.ke, g.j3oj2, g.vkms,
        double(c.resonant), c.dedt, c.didt, c.dMdt, c.dnodedt, c.dargpdt, c.Mbody0[0], c.Mbody0[1],
        c.pe2[0], c.pe3[0], c.pi2[0], c.pi3[0], c.pl2[0], c.pl3[0], c.pl4[0], c.pgh2[0], c.pgh3[0], c.pgh4[0],
        c.ph2[0], c.ph3[0],
        c.pe2[1], c.pe3[1], c.pi2[1], c.pi3[1], c.pl2[1], c.pl3[1], c.pl4[1], c.pgh2[1], c.pgh3[1], c.pgh4[1],
        c.ph2[1], c.ph3[1],
        double(c.irez), c.xlamo, c.xfact, c.gsto,
        c.res[0], c.res[1], c.res[2], c.res[3], c.res[4], c.res[5], c.res[6], c.res[7], c.res[8], c.res[9]};
    static_assert(sizeof out == kI_COUNT * sizeof(double), "init export");
    std::memcpy(rec + i * kI_COUNT, out, sizeof out);
  }
  return 0;
}

// Resonance internals, for the pins.  Inclination and eccentricity functions
// at (e, i): out[0..11] F in the order F311 F220 F330 F221 F321 F322 F441 F442
// F522 F523 F542 F543, out[12..24] G in the order G310 (24 h series) G200 G300
// G201 G211 G310 G322 G410 G422 G520 G532 G521 G533.
void oracle_resonance_functions(double e, double inc, double* out) {
  double F[kNF], G[kNG];
  res_inclination(std::cos(inc), std::sin(inc), F);
  res_eccentricity(e, G);
  for (int k = 0; k < kNF; ++k) out[k] = F[k];
  for (int k = 0; k < kNG; ++k) out[kNF + k] = G[k];
}

// Model constants: out[0] the Earth's rotation rate (rad/min), out[1] the
// step (min), then per term (24 h: 3, then 12 h: 10) j, k, l, phase, J.
int oracle_resonance_constants(double* out) {
  out[0] = kEarthRate;
  out[1] = kResStep;
  int m = 2;
  for (const ResTerm& q : kRes24) { out[m++] = q.j; out[m++] = q.k; out[m++] = q.l; out[m++] = q.phase; out[m++] = q.J; }
  for (const ResTerm& q : kRes12) { out[m++] = q.j; out[m++] = q.k; out[m++] = q.l; out[m++] = q.phase; out[m++] = q.J; }
  return m;
}

// Sidereal angle (rad) at a Julian date taken as UT1.
double oracle_gmst(double jd) { return gmst_iau82(jd - 2415020.0); }

// For one element set elem1[8] (the current reference date applies): the
// rates (dn/dt, d2n/dt2, dlambda/dt) at (xli, xni, atime), and the integrated
// (lambda, n, time of the last step) at t minutes after epoch.  Return the
// resonance class (0 when the set is not resonant; nothing written).
int oracle_resonance_rates(const double* grav, const double* elem1, double xli, double xni, double atime,
                           double* out3) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  double el[kNElem];
  for (int k = 0; k < kNElem; ++k) el[k] = elem1[k];
  Sat<double> c = sgp4_init<double>(g, el, elem1[7]);
  if (!c.irez) return 0;
  res_rates(c, xli, xni, atime, &out3[0], &out3[1], &out3[2]);
  return c.irez;
}
int oracle_resonance_integrate(const double* grav, const double* elem1, double t, double* out3) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  double el[kNElem];
  for (int k = 0; k < kNElem; ++k) el[k] = elem1[k];
  Sat<double> c = sgp4_init<double>(g, el, elem1[7]);
  if (!c.irez) return 0;
  out3[2] = res_integrate(c, t, &out3[0], &out3[1]);
  return c.irez;
}

// Forward-mode Jacobian d(r, v)/d(n0, e0, i0, node0, argp0, M0, bstar) at
// individual points: J[k][6][7] (rows rx ry rz vx vy vz).
int oracle_jacobian_points(const double* grav, int64_t n, const double* elem, int64_t npts, const int64_t* sat,
                           const double* t, double* J, double* r, double* v, uint8_t* err) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  for (int64_t k = 0; k < npts; ++k) {
    if (sat[k] < 0 || sat[k] >= n) return -1;
    Dual el[kNElem];
    double epoch;
    load_elements(elem, n, sat[k], el, &epoch);
    for (int q = 0; q < kNElem; ++q) el[q].d[q] = 1.0;
    Sat<Dual> c = sgp4_init<Dual>(g, el, epoch);
    Dual rr[3], vv[3];
    int code = sgp4_point(g, c, t[k] - 1440.0 * epoch, rr, vv, nullptr);
    for (int q = 0; q < 3; ++q) {
      r[q * npts + k] = rr[q].v; v[q * npts + k] = vv[q].v;
      for (int m = 0; m < kNElem; ++m) {
        J[(k * 6 + q) * kNElem + m] = rr[q].d[m];
        J[(k * 6 + 3 + q) * kNElem + m] = vv[q].d[m];
      }
    }
    err[k] = uint8_t(code);
  }
  return 0;
}

// Vector-Jacobian product over a dense n x T grid: gelem[7][n] =
// sum_j sum_c gr[c][i*T+j] dr_c/dtheta + gv[c][i*T+j] dv_c/dtheta, with gv
// nullable (zero).  Points with codes 1, 2, 4, 7 contribute nothing.
int oracle_vjp(const double* grav, int64_t n, const double* elem, const double* t, int64_t T, const double* gr,
               const double* gv, double* gelem, int nthreads) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  const int64_t P = n * T;
  parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      Dual el[kNElem];
      double epoch;
      load_elements(elem, n, i, el, &epoch);
      for (int q = 0; q < kNElem; ++q) el[q].d[q] = 1.0;
      Sat<Dual> c = sgp4_init<Dual>(g, el, epoch);
      double acc[kNElem] = {0};
      for (int64_t j = 0; j < T; ++j) {
        Dual rr[3], vv[3];
        int code = sgp4_point(g, c, t[j] - 1440.0 * epoch, rr, vv, nullptr);
        if (code != 0 && code != 6) continue;
        const int64_t p = i * T + j;
        for (int q = 0; q < 3; ++q)
          for (int m = 0; m < kNElem; ++m) {
            acc[m] += gr[q * P + p] * rr[q].d[m];
            if (gv) acc[m] += gv[q * P + p] * vv[q].d[m];
          }
      }
      for (int m = 0; m < kNElem; ++m) gelem[m * n + i] = acc[m];
    }
  });
  return 0;
}

// Vector-Jacobian product over CSR time lists: satellite i's points are
// offsets[i] .. offsets[i+1]-1, at times t[p]; gelem[7][n] as for oracle_vjp
// with the cotangent rows gr[c][p], gv[c][p] (gv nullable).
int oracle_vjp_ragged(const double* grav, int64_t n, const double* elem, const int64_t* offsets, const double* t,
                      int64_t nnz, const double* gr, const double* gv, double* gelem, int nthreads) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  if (n < 0 || nnz < 0 || offsets[0] != 0 || offsets[n] != nnz) return -3;
  for (int64_t i = 0; i < n; ++i) if (offsets[i + 1] < offsets[i]) return -3;
  parallel_for(n, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      Dual el[kNElem];
      double epoch;
      load_elements(elem, n, i, el, &epoch);
      for (int q = 0; q < kNElem; ++q) el[q].d[q] = 1.0;
      Sat<Dual> c = sgp4_init<Dual>(g, el, epoch);
      double acc[kNElem] = {0};
      for (int64_t p = offsets[i]; p < offsets[i + 1]; ++p) {
        Dual rr[3], vv[3];
        int code = sgp4_point(g, c, t[p] - 1440.0 * epoch, rr, vv, nullptr);
        if (code != 0 && code != 6) continue;
        for (int q = 0; q < 3; ++q)
          for (int m = 0; m < kNElem; ++m) {
            acc[m] += gr[q * nnz + p] * rr[q].d[m];
            if (gv) acc[m] += gv[q * nnz + p] * vv[q].d[m];
          }
      }
      for (int m = 0; m < kNElem; ++m) gelem[m * n + i] = acc[m];
    }
  });
  return 0;
}

// Arithmetic the definition performs for one point (initialisation excluded):
// out[8] = {add/sub, mul, div, sqrt, cbrt, sin/cos, atan2, floor}.
int oracle_count_ops(const double* grav, const double* elem1 /*[8]*/, double tmin, uint64_t* out8) {
  Gravity g;
  if (int rc = make_gravity(grav, &g)) return rc;
  OpCount el[kNElem];
  for (int k = 0; k < kNElem; ++k) el[k] = OpCount(elem1[k]);
  Sat<OpCount> c = sgp4_init<OpCount>(g, el, elem1[7]);
  g_tally = OpTally();
  OpCount rr[3], vv[3];
  int code = sgp4_point(g, c, tmin - 1440.0 * elem1[7], rr, vv, nullptr);
  uint64_t o[8] = {g_tally.add, g_tally.mul, g_tally.div, g_tally.sqrt, g_tally.cbrt, g_tally.trig, g_tally.atan2, g_tally.floor};
  std::memcpy(out8, o, sizeof o);
  return code;
}

}  // extern "C"

// Per-point SGP4 near-Earth propagation, templated on precision.
//
// One lane evaluates f(s, t) -> (r, v) for one (satellite, time) point, all in
// registers (paper section 2.2: the whole routine fused, with validity checks
// turned into per-point codes instead of early exits of the batch).  The
// steps follow the published near-Earth model: secular gravity and drag,
// long-period (J3) periodics, Kepler's equation for the eccentric longitude,
// short-period (J2) periodics, orientation and the TEME state in km, km/s.
//
// Precision policy (TS = secular type, TP = periodic type):
//   FP64        TS = double, TP = double
//   FP32 plain  TS = float,  TP = float   (time since epoch rounded to float:
//               the paper's 32-bit mode, section 4)
//   FP32 mixed  TS = double, TP = float   (time since epoch, the n*t and drag
//               polynomials, the angle sums and their reduction mod 2*pi in
//               double; everything after the reduction in float)
#pragma once

#include "sgp4mi_common.h"
#include "sgp4mi_math.h"

namespace sgp4mi {

template <class TS, class TP>
struct SatC {
  // secular (TS)
  TS M0, Mdot, argp0, argpdot, node0, nodedot, nodecf, C1, bC4, t2cof, argpcof, Mcof, D2, D3, D4, bC5;
  TS t3cof, t4cof, t5cof, n0pp, a0pp, e0;
  double epoch_min;
  // periodic (TP)
  TP eta, dM0, sinM0, aycof, Lcof, c41, x1, x7, cosi, sini, i0;
  TP spA1, spX1h, spX1k, spX7q, spCN, spCI;
  // the drag constants again in TP: near-Earth propagation evaluates the drag
  // polynomials in the periodic type (the mean-anomaly polynomial excepted)
  TP pC1, pbC4, pD2, pD3, pD4, pbC5, pMcof, pArgpcof, pA0pp, pE0;
  uint32_t info;
  const double* deep;  // the deep-space slot's entries (read only when info has kInfoDeep)
};

// Global-address-space view of a slot, for loads the compiler keeps as
// global (not flat) vector loads.
typedef const __attribute__((address_space(1))) Slot* GSlot;

// The slot address seen as a per-lane value: loads through it are vector
// loads into VGPRs (one broadcast fetch per wavefront when every lane holds the
// same satellite) instead of scalar loads into SGPRs.  With ~34 constants per
// satellite, SGPR residency overflows the scalar file and every VALU operation
// reading two of them needs an extra move; VGPR residency has neither cost.
__device__ __forceinline__ GSlot lane_slot(const Slot* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  uint32_t lo = uint32_t(v), hi = uint32_t(v >> 32);
  asm volatile("v_mov_b32 %0, %0" : "+v"(lo));
  asm volatile("v_mov_b32 %0, %0" : "+v"(hi));
  return (GSlot)((uint64_t(hi) << 32) | lo);
}

// Constant-address-space view of a slot.  The record is never written while a
// propagation kernel runs; loads through this view stay scalar loads even
// after the kernel's own stores, which the compiler cannot otherwise prove do
// not alias the record (a wavefront that stores and then reads the next
// point's constants would get vector loads into VGPRs).
typedef const __attribute__((address_space(4))) Slot* CSlot;

template <class T, class P> __device__ __forceinline__ T rec_val(P sp, int k);
template <> __device__ __forceinline__ double rec_val<double, const Slot*>(const Slot* sp, int k) { return sp->d[k]; }
template <> __device__ __forceinline__ float rec_val<float, const Slot*>(const Slot* sp, int k) { return sp->f[k]; }
template <> __device__ __forceinline__ double rec_val<double, GSlot>(GSlot sp, int k) { return sp->d[k]; }
template <> __device__ __forceinline__ float rec_val<float, GSlot>(GSlot sp, int k) { return sp->f[k]; }
template <> __device__ __forceinline__ double rec_val<double, CSlot>(CSlot sp, int k) { return sp->d[k]; }
template <> __device__ __forceinline__ float rec_val<float, CSlot>(CSlot sp, int k) { return sp->f[k]; }

// Secular constants (and the info word) through sp, periodic constants
// through pp (the same slot, possibly seen through another address space).
template <class TS, class TP, class P, class PP>
__device__ __forceinline__ SatC<TS, TP> load_from(P sp, PP pp) {
  SatC<TS, TP> c;
#define S_(k) rec_val<TS, P>(sp, k)
#define P_(k) rec_val<TP, PP>(pp, k)
  c.M0 = S_(kM0); c.Mdot = S_(kMdot); c.argp0 = S_(kArgp0); c.argpdot = S_(kArgpdot); c.node0 = S_(kNode0);
  c.nodedot = S_(kNodedot); c.nodecf = S_(kNodecf); c.C1 = S_(kC1); c.bC4 = S_(kBC4); c.t2cof = S_(kT2cof);
  c.argpcof = S_(kArgpcof); c.Mcof = S_(kMcof); c.D2 = S_(kD2); c.D3 = S_(kD3); c.D4 = S_(kD4); c.bC5 = S_(kBC5);
  c.t3cof = S_(kT3cof); c.t4cof = S_(kT4cof); c.t5cof = S_(kT5cof); c.n0pp = S_(kN0pp); c.a0pp = S_(kA0pp);
  c.e0 = S_(kE0);
  c.epoch_min = rec_val<double, P>(sp, kEpochMin);
  c.eta = P_(kEta); c.dM0 = P_(kDM0); c.sinM0 = P_(kSinM0); c.aycof = P_(kAycof); c.Lcof = P_(kLcof);
  c.c41 = P_(kC41); c.x1 = P_(kX1); c.x7 = P_(kX7); c.cosi = P_(kCosi); c.sini = P_(kSini); c.i0 = P_(kI0);
  c.spA1 = P_(kSpA1); c.spX1h = P_(kSpX1h); c.spX1k = P_(kSpX1k); c.spX7q = P_(kSpX7q); c.spCN = P_(kSpCN);
  c.spCI = P_(kSpCI);
  c.pC1 = P_(kC1); c.pbC4 = P_(kBC4); c.pD2 = P_(kD2); c.pD3 = P_(kD3); c.pD4 = P_(kD4); c.pbC5 = P_(kBC5);
  c.pMcof = P_(kMcof); c.pArgpcof = P_(kArgpcof); c.pA0pp = P_(kA0pp); c.pE0 = P_(kE0);
#undef S_
#undef P_
  c.info = sp->info;
  return c;
}

template <class TS, class TP, bool kVec>
__device__ __forceinline__ SatC<TS, TP> load_sat(const RecordView& rv, int64_t i) {
  SatC<TS, TP> c;
  if (kVec) {
    const GSlot v = lane_slot(rv.slots + i);
    c = load_from<TS, TP, GSlot, GSlot>(v, v);
  } else {
    const CSlot cp = (CSlot)(rv.slots + i);
    c = load_from<TS, TP, CSlot, CSlot>(cp, cp);
  }
  c.deep = rv.deep[i].d;
  return c;
}

__device__ __forceinline__ Grav load_grav(const RecordView& rv) {
  Grav g;
  typedef const __attribute__((address_space(4))) double* CHdr;  // read-only while kernels run
  const CHdr h = (CHdr)rv.hdr;
  g.ke = h[kHKe];
  g.radius = h[kHRadius];
  g.vkms = h[kHVkms];
  g.k2 = h[kHK2];
  g.j3oj2 = h[kHJ3oJ2];
  const __attribute__((address_space(4))) float* f = (const __attribute__((address_space(4))) float*)(h + kHF32);
  g.radius_f = f[0];
  g.vkms_f = f[1];
  g.k2_f = f[2];
  return g;
}

// ------------------------------------------------------- typed primitives --
// Sine and cosine of an angle held in the secular type, evaluated in the
// periodic type (reduction in the secular type).  sc_damped serves angles whose
// sine and cosine enter the state only through a small factor (the
// eccentricity in e cos w, e sin w; the drag coefficients multiplying
// functions of M).  In the mixed path every angle goes to the 32-bit hardware
// sine and cosine (argument reduced to a turn fraction in double; absolute
// error ~1.3e-7, a few tenths of a metre at LEO radius); the plain FP32 path
// keeps its series for the undamped angles, FP64 its series everywhere.
template <class TS, class TP>
struct Trig;
template <>
struct Trig<double, double> {
  static __device__ __forceinline__ void sc(double x, double* s, double* c) { sincos_rr(x, s, c); }
  static __device__ __forceinline__ void sc_damped(double x, double* s, double* c) { sincos_rr(x, s, c); }
};
template <>
struct Trig<float, float> {
  static __device__ __forceinline__ void sc(float x, float* s, float* c) { sincos_rr(x, s, c); }
  static __device__ __forceinline__ void sc_damped(float x, float* s, float* c) { sincos_hw(x, s, c); }
};
template <>
struct Trig<double, float> {
  static __device__ __forceinline__ void sc(double x, float* s, float* c) { sincos_hw(x, s, c); }
  static __device__ __forceinline__ void sc_damped(double x, float* s, float* c) { sincos_hw(x, s, c); }
};

__device__ __forceinline__ double wrap(double x) { return wrap_pi(x); }
__device__ __forceinline__ float wrap(float x) {
  return fmaf(-6.28318530717958647692f, rintf(x * 0.15915494309189533577f), x);
}
__device__ __forceinline__ double sq_root(double x) { return sqrt(x); }
__device__ __forceinline__ float sq_root(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// a + b t for per-satellite constants a and b.  Double keeps the product and
// the sum apart: fused, the instruction would read both constants from scalar
// registers, one more than it can take, and a two-register move would come
// first.  Float fuses (one move of one register).
__device__ __forceinline__ double lin(double a, double b, double t) {
#pragma clang fp contract(off)
  return a + b * t;
}
__device__ __forceinline__ float lin(float a, float b, float t) { return fmaf(b, t, a); }
__device__ __forceinline__ double vfma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float vfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double vmax(double x, double y) { return fmax(x, y); }
__device__ __forceinline__ float vmax(float x, float y) { return fmaxf(x, y); }
__device__ __forceinline__ double vabs(double x) { return fabs(x); }
__device__ __forceinline__ float vabs(float x) { return fabsf(x); }
__device__ __forceinline__ double arctan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float arctan2(float y, float x) { return atan2f(y, x); }
// Kepler tolerance: the model's 1e-12 in double; in float the eccentric
// longitude offset is resolved to ~1e-10, so 1e-7 rad (sub-millimetre) ends it.
template <class T> __device__ __forceinline__ T kepler_tol();
template <> __device__ __forceinline__ double kepler_tol<double>() { return 1.0e-12; }
template <> __device__ __forceinline__ float kepler_tol<float>() { return 1.0e-7f; }

// Newton step clamped to [-0.95, 0.95] (one median-of-three in float).  A NaN
// step (possible only when e_L >= 1, where the point's code is 4 and its state
// is not used) comes out finite here.  hi = 0.95 comes from step_bound: in
// float it is held in a vector register for the whole iteration (the
// median-of-three takes at most one scalar-register operand), instead of a
// move per step.
template <class T> __device__ __forceinline__ T step_bound();
template <> __device__ __forceinline__ double step_bound<double>() { return 0.95; }
template <> __device__ __forceinline__ float step_bound<float>() {
  float x = 0.95f;
  asm("" : "+v"(x));
  return x;
}
__device__ __forceinline__ double clamp_step(double x) { return fmax(fmin(x, 0.95), -0.95); }
__device__ __forceinline__ float clamp_step(float x) { return __builtin_amdgcn_fmed3f(x, -0.95f, 0.95f); }
__device__ __forceinline__ double clamp_step(double x, double hi) { return fmax(fmin(x, hi), -hi); }
__device__ __forceinline__ float clamp_step(float x, float hi) {
  return __builtin_amdgcn_fmed3f(x, sgpr_const(-0.95f), hi);
}

// Kepler exit test for a step of size as (see the iteration in sgp4_point):
// as < tol, or quad * as^2 < tol with quad = eb while eb < 1/2.  Double
// evaluates it as written.  Float folds both into one comparison with a
// per-point threshold, as < max(tol, sqrt(tol / eb)) while eb < 1/2, else
// as < tol (the same test up to the rounding of the threshold, which can
// only decide whether a step of about the tolerance is taken).
template <class TP> struct KeplerExit;
template <> struct KeplerExit<double> {
  double quad;
  __device__ __forceinline__ explicit KeplerExit(double eb) : quad(eb < 0.5 ? eb : 1.0e30) {}
  __device__ __forceinline__ bool operator()(double as) const {
    return as < kepler_tol<double>() || quad * as * as < kepler_tol<double>();
  }
};
template <> struct KeplerExit<float> {
  float thr;
  __device__ __forceinline__ explicit KeplerExit(float eb) {
    const float t = __builtin_sqrtf(kepler_tol<float>()) * rsq(eb);  // sqrt(tol / eb); the root folds to a constant
    thr = fmaxf(eb < 0.5f ? t : 0.0f, kepler_tol<float>());
  }
  __device__ __forceinline__ bool operator()(float as) const { return as < thr; }
};

// ok: whether r and v hold a state (codes 0 and 6).  Set from the control
// flow, it stays a lane mask in scalar registers: the writer branches on it
// without comparing the code.
template <class TP>
struct PointState {
  TP r[3], v[3];
  bool ok;
};

// Inclination functions and J3 coefficients the periodic terms use: the
// epoch's (per-satellite constants) in near-Earth propagation, the
// lunar-solar perturbed ones (per point) in deep space.  The float paths
// take the short-period coefficients with k2 = J2 / 2 folded in: A1 = 1.5 k2
// (3 cos^2 i - 1), X1h = k2 / 2 sin^2 i, X1k = k2 sin^2 i, X7q = -k2 / 4
// (7 cos^2 i - 1), CN = 1.5 k2 cos i, CI = 1.5 k2 cos i sin i (fewer
// instructions per point, each reading at most one of them); FP64 multiplies
// by k2 per point (its constants are register pairs, and six more would
// overflow the scalar register file).
template <class TS, class TP>
struct Incl {
  TP c41, x1, x7, cosi, sini, i0, aycof, Lcof;
  TP A1, X1h, X1k, X7q, CN, CI;
};

// Long-period (J3) and short-period (J2) periodics, Kepler's equation,
// orientation and the TEME state, from the mean elements a, e (already
// floored) and the angles M, argp, node (unreduced).  Returns 0, 4 or 6.
//
// Reformulations relative to the textbook order, each an identity up to
// rounding: the Kepler iteration carries psi - U and rotates (sin psi,
// cos psi) by each Newton step; the argument of latitude u never leaves its
// (sin, cos) pair (no atan2: the short-period correction is a rotation of the
// normalised pair); sin/cos of the corrected inclination rotate those of i0.
// Rotations fall back to a full evaluation when the angle exceeds kRotMax.
template <class TS, class TP>
__device__ __forceinline__ uint32_t sgp4_tail(const Grav& g, TP a, TP e, TS M, TS argp, TS node,
                                              const Incl<TS, TP>& q, PointState<TP>& out) {
  using TR = Trig<TS, TP>;
  // Long-period periodics (J3).
  TP sw, cw;
  TR::sc_damped(argp, &sw, &cw);
  const TP axn = e * cw;
  const TP tau = rcp(a * (TP(1) - e * e));
  const TP ayn = e * sw + tau * q.aycof;

  // Kepler: psi - axn sin psi + ayn cos psi = U, Newton from psi = U with the
  // step clamped to +-0.95; dpsi = psi - U.  A lane is done once its step is
  // below the tolerance or once a bound on the next step is: Newton's next
  // step is at most eL / (2 (1 - eL)) * step^2 with eL <= |axn| + |ayn|, itself
  // at most eL * step^2 while eL < 1/2 (so the step that would follow changes
  // psi by less than the tolerance).  The loop ends when every lane of the
  // wavefront is done (at most 10 steps).
  // U = L_T - node, with the mean longitude L = M + argp + node and its J3
  // long-period correction L_T = L + tau L_cof a_xN: node cancels.
  const TS U = M + argp + TS(tau * q.Lcof * axn);
  TP sp, cp;
  TR::sc(U, &sp, &cp);
  TP dpsi = TP(0);
  const TP eb = vabs(axn) + vabs(ayn);
  const KeplerExit<TP> done(eb);
  const TP hi = step_bound<TP>();
  for (int k = 0; k < 10; ++k) {
    TP step = (axn * sp - ayn * cp - dpsi) * rcp(TP(1) - axn * cp - ayn * sp);
    step = clamp_step(step, hi);
    dpsi = sizeof(TP) == 4 && k == 0 ? step : dpsi + step;  // float: no 0 + step
    if (vabs(step) <= TP(kRotMax)) rotate_small(&sp, &cp, step);
    else TR::sc(U + TS(dpsi), &sp, &cp);
    if (__all(done(vabs(step)))) break;
  }

  // Short-period preliminaries.
  const TP ecE = axn * cp + ayn * sp;
  const TP esE = axn * sp - ayn * cp;
  const TP eL2 = axn * axn + ayn * ayn;
  const TP pL = a * (TP(1) - eL2);
  if (!(pL >= TP(0))) return 4;
  const TP rl = a * (TP(1) - ecE);
  const TP inv_rl = rcp(rl);
  const TP ra = rsq(a);
  const TP sqa = a * ra;
  const TP rdotl = sqa * esE * inv_rl;
  const TP betal = sq_root(TP(1) - eL2);
  const TP rvdotl = sqa * betal * inv_rl;  // sqrt(pL) = sqrt(a) * sqrt(1 - eL^2)
  const TP w = esE * rcp(TP(1) + betal);
  const TP ar = a * inv_rl;
  const TP sinu = ar * (sp - ayn - axn * w);
  const TP cosu = ar * (cp - axn + ayn * w);
  const TP sin2u = TP(2) * sinu * cosu;
  const TP cos2u = TP(1) - TP(2) * sinu * sinu;

  // Short-period periodics (J2).
  const TP inv_pl = rcp(pL);
  const TP nk = ra * ra * ra;  // n / ke = a^-3/2
  TP mrt, du, dnode, dinc, mvt, rvdot;
  if (sizeof(TP) == 4) {
    // k2 / p_L and k2 / p_L^2 times the inclination functions, k2 in the
    // coefficients
    const TP ip2 = inv_pl * inv_pl;
    const TP ni = nk * inv_pl;
    const TP s2 = ip2 * sin2u, c2 = ip2 * cos2u;
    mrt = rl * vfma(-ip2 * betal, q.A1, TP(1)) + inv_pl * cos2u * q.X1h;
    du = q.X7q * s2;
    dnode = q.CN * s2;
    dinc = q.CI * c2;
    mvt = rdotl - ni * sin2u * q.X1k;
    rvdot = rvdotl + ni * vfma(q.X1k, cos2u, q.A1);
  } else {
    const TP k1 = grav_k2<TP>(g) * inv_pl;
    const TP k2 = k1 * inv_pl;
    // 1.5 c41 as c41 + c41 / 2 (one instruction reading one scalar register
    // twice; 1.5 is no inline constant); the same single rounding of 1.5 c41
    const TP c41h = vfma(q.c41, TP(0.5), q.c41);
    mrt = rl * (TP(1) - k2 * betal * c41h) + TP(0.5) * k1 * q.x1 * cos2u;
    du = TP(-0.25) * k2 * q.x7 * sin2u;
    dnode = TP(1.5) * k2 * q.cosi * sin2u;
    dinc = TP(1.5) * k2 * q.cosi * q.sini * cos2u;
    mvt = rdotl - nk * k1 * q.x1 * sin2u;
    rvdot = rvdotl + nk * k1 * vfma(q.x1, cos2u, c41h);
  }

  // Orientation: sin/cos of u_k = u + du, i_k = i0 + dinc, node_k = node + dnode.
  TP ssu, csu;
  if (vabs(du) <= TP(kRotMax)) {
    // (sinu, cosu) is a unit vector up to rounding; one Newton step from 1
    // normalises it to O(delta^2), delta = |.|^2 - 1 (float rounding leaves
    // delta ~1e-6 at most, so the float paths need no other case)
    const TP n2 = sinu * sinu + cosu * cosu;
    TP h = TP(1.5) - TP(0.5) * n2;
    if (sizeof(TP) == 8 && vabs(n2 - TP(1)) > TP(1.0e-8)) h = rsq(n2);
    ssu = sinu * h;
    csu = cosu * h;
    rotate_small(&ssu, &csu, du);
  } else {
    TR::sc(TS(arctan2(sinu, cosu) + du), &ssu, &csu);
  }
  TP sinc = q.sini, cinc = q.cosi;
  if (vabs(dinc) <= TP(kRotMax)) rotate_small(&sinc, &cinc, dinc);
  else TR::sc(TS(q.i0 + dinc), &sinc, &cinc);
  TP snod, cnod;
  TR::sc(node + TS(dnode), &snod, &cnod);

  const TP xmx = -snod * cinc, xmy = cnod * cinc;
  const TP ux = xmx * ssu + cnod * csu, uy = xmy * ssu + snod * csu, uz = sinc * ssu;
  const TP vx = xmx * csu - cnod * ssu, vy = xmy * csu - snod * ssu, vz = sinc * csu;
  const TP rk = mrt * grav_radius<TP>(g);
  const TP vk = grav_vkms<TP>(g);
  out.r[0] = rk * ux; out.r[1] = rk * uy; out.r[2] = rk * uz;
  out.v[0] = vk * (mvt * ux + rvdot * vx);
  out.v[1] = vk * (mvt * uy + rvdot * vy);
  out.v[2] = vk * (mvt * uz + rvdot * vz);
  out.ok = true;
  return (mrt < TP(1)) ? 6u : 0u;
}


// Tesseral resonance of the 24 h and 12 h classes: the mean motion and the
// resonant mean longitude integrated from epoch in steps of 720 minutes
// toward t while a whole step remains (second-order Taylor steps), then the
// Taylor polynomial over the remainder; the integrator's state in double in
// every path.  Rates at (lambda, n, w): dn/dt = sum of a sin A - b cos A over
// the terms, A = j w + k lambda and (a, b) the term's coefficient times the
// cosine and sine of its phase; d2n/dt2 = dlambda/dt times the sum of k (a cos
// A + b sin A); dlambda/dt = n + the rest of the argument's secular rate.
// TR: the type the rates are evaluated in.  The float paths take them in
// float (hardware sine and cosine of the angle reduced in double): a relative
// error of ~1e-7 in dn/dt, ~1e-11 rad/min^2, moves lambda by ~1e-9 rad over a
// week, far below the float state's own rounding.
template <class TR>
__device__ __forceinline__ void res_rates(bool sync24, const double* d, double xli, double w, double xni,
                                          double* ndot, double* nddot, double* ldot) {
  const double* r = d + kDRc0;
  TR s1, c1;
  if constexpr (sizeof(TR) == 8)
    sincos_rr(xli, &s1, &c1);
  else
    sincos_hw(xli, &s1, &c1);
  const TR s2 = TR(2) * s1 * c1, c2 = TR(1) - TR(2) * s1 * s1;
  TR sn, cs;
  if (sync24) {
    // 24 h: A = lambda, 2 lambda, 3 lambda
    const TR s3 = s1 * (TR(3) - TR(4) * s1 * s1), c3 = c1 * (TR(4) * c1 * c1 - TR(3));
    sn = (TR(r[0]) * s1 - TR(r[1]) * c1) + (TR(r[2]) * s2 - TR(r[3]) * c2) + (TR(r[4]) * s3 - TR(r[5]) * c3);
    cs = (TR(r[0]) * c1 + TR(r[1]) * s1) + TR(2) * (TR(r[2]) * c2 + TR(r[3]) * s2) +
         TR(3) * (TR(r[4]) * c3 + TR(r[5]) * s3);
  } else {
    // 12 h: (j, k) = (2,1) (0,1) (1,1) (-1,1) (2,2) (0,2) (1,1) (-1,1) (1,2)
    // (-1,2); the third and seventh terms, and the fourth and eighth, share
    // their angle
    TR sw, cw;
    if constexpr (sizeof(TR) == 8)
      sincos_rr(w, &sw, &cw);
    else
      sincos_hw(w, &sw, &cw);
    const TR sw2 = TR(2) * sw * cw, cw2 = TR(1) - TR(2) * sw * sw;
    TR s1x = TR(0), c1x = TR(0), s2x = TR(0), c2x = TR(0);  // k = 1 and k = 2 sums
    auto term = [&](double a, double b, TR sA, TR cA, TR* sk, TR* ck) {
      *sk += TR(a) * sA - TR(b) * cA;
      *ck += TR(a) * cA + TR(b) * sA;
    };
    term(r[0], r[1], sw2 * c1 + cw2 * s1, cw2 * c1 - sw2 * s1, &s1x, &c1x);
    term(r[2], r[3], s1, c1, &s1x, &c1x);
    term(r[4] + r[12], r[5] + r[13], sw * c1 + cw * s1, cw * c1 - sw * s1, &s1x, &c1x);
    term(r[6] + r[14], r[7] + r[15], s1 * cw - c1 * sw, c1 * cw + s1 * sw, &s1x, &c1x);
    term(r[8], r[9], sw2 * c2 + cw2 * s2, cw2 * c2 - sw2 * s2, &s2x, &c2x);
    term(r[10], r[11], s2, c2, &s2x, &c2x);
    term(r[16], r[17], sw * c2 + cw * s2, cw * c2 - sw * s2, &s2x, &c2x);
    term(r[18], r[19], s2 * cw - c2 * sw, c2 * cw + s2 * sw, &s2x, &c2x);
    sn = s1x + s2x;
    cs = c1x + TR(2) * c2x;
  }
  *ldot = xni + d[kDXfact];
  *ndot = double(sn);
  *nddot = double(cs) * *ldot;
}

// Integrated (lambda, n) at t minutes after epoch; NaN beyond 10 years from
// epoch or for t not finite (every lane's loop is bounded by that reach).
template <class TR>
__device__ __forceinline__ void res_integrate(bool sync24, const double* d, double t, double n0, double argp0,
                                              double argpdot, double* xl, double* nm) {
  if (!(fabs(t) <= kResMaxMin)) {
    *xl = *nm = __builtin_nan("");
    return;
  }
  double xli = d[kDXlamo], xni = n0, atime = 0.0, ndot, nddot, ldot;
  const double h = t > 0.0 ? kResStepMin : -kResStepMin;
  const double hh = 0.5 * h * h;
  for (;;) {
    res_rates<TR>(sync24, d, xli, argp0 + argpdot * atime, xni, &ndot, &nddot, &ldot);
    if (!(fabs(t - atime) >= kResStepMin)) break;
    xli = xli + ldot * h + ndot * hh;
    xni = xni + ndot * h + nddot * hh;
    atime += h;
  }
  const double ft = t - atime;
  *nm = xni + ndot * ft + nddot * (0.5 * ft * ft);
  *xl = xli + ldot * ft + ndot * (0.5 * ft * ft);
}

// Deep space (period of 225 min or more): the near-Earth
// secular terms with the simplified drag, the lunar-solar secular rates, for
// the resonant classes the integrated mean motion and the mean anomaly from
// the resonant longitude, then the Sun's and the Moon's long-period terms on
// the mean elements (each body's
// mean anomaly advanced by its mean motion, its true anomaly to first order in
// its eccentricity); below 0.2 rad of perturbed inclination the node and
// inclination changes are applied to (sin i sin node, sin i cos node) and the
// longitude argp + cos i node is carried instead, so nothing divides by
// sin i.  The inclination functions of the periodic terms follow the
// perturbed inclination.  All of this in the secular type; code 3 when the
// perturbed eccentricity leaves [0, 1].
template <class TS, class TP>
__device__ __forceinline__ uint32_t deep_point(const SatC<TS, TP>& c, const Grav& g, double t_abs,
                                            PointState<TP>& out) {
  out.ok = false;
  const uint32_t scode = c.info & kInfoCodeMask;  // codes 1, 2 at epoch
  if (scode) return scode;
  const double* d = c.deep;
  const TS t = TS(t_abs - c.epoch_min);
  const TS t2 = t * t;
  TS M = lin(c.M0, c.Mdot, t) + TS(d[kDMDt]) * t;
  TS argp = lin(c.argp0, c.argpdot, t) + TS(d[kDArgpDt]) * t;
  TS node = lin(c.node0, c.nodedot, t) + c.nodecf * t2 + TS(d[kDNodeDt]) * t;
  const TS incl = TS(c.i0) + TS(d[kDiDt]) * t;
  const TS A = TS(1) - c.C1 * t;
  TS a0 = c.a0pp;
  const double rcls = d[kDRes];
  if (rcls != 0.0) {
    // resonance: M from the resonant longitude and the sidereal angle at t,
    // a from the integrated mean motion (code 2 if it is not positive)
    const double td = t_abs - c.epoch_min;
    double xl, nm;
    res_integrate<TP>(rcls == 1.0, d, td, double(c.n0pp), double(c.argp0), double(c.argpdot), &xl, &nm);
    const double th = d[kDGsto] + td * kEarthRot;
    const double theta = th - kTwoPi * floor(th * kInvTwoPi);
    if (rcls == 1.0)
      M = TS(xl) - node - argp + TS(theta);
    else
      M = TS(xl) - TS(2) * node + TS(2) * TS(theta);
    if (!(nm > 0.0)) return 2;
    const double cr = cbrt(g.ke / nm);
    a0 = TS(cr * cr);
  }
  const TS a_s = a0 * A * A;
  TS e = c.e0 + TS(d[kDeDt]) * t - c.bC4 * t;
  if (!(e >= TS(-0.001) && e < TS(1))) return 1;
  e = vmax(e, TS(1.0e-6));
  M = M + c.n0pp * (c.t2cof * t2);
  // mean longitude; angles reduced to [0, 2 pi) (the low-inclination form
  // uses the node's value)
  const TS twopi = TS(kTwoPi), itwopi = TS(kInvTwoPi);
  TS L = M + argp + node;
  node = node - twopi * floor(node * itwopi);
  argp = argp - twopi * floor(argp * itwopi);
  L = L - twopi * floor(L * itwopi);
  M = L - argp - node;
  // lunar and solar long-period terms
  TS pe = TS(0), pinc = TS(0), pl = TS(0), pgh = TS(0), ph = TS(0);
  const double nb[2] = {1.19459e-5, 1.5835218e-4}, eb[2] = {0.01675, 0.05490};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double* q = d + kDPer0 + kNPer * k;
    const TS Mb = TS(d[kDMb0 + k]) + TS(nb[k]) * t;
    TS sMb, cMb;
    Trig<TS, TS>::sc(Mb, &sMb, &cMb);
    TS sf, cf;
    Trig<TS, TS>::sc(Mb + TS(2.0 * eb[k]) * sMb, &sf, &cf);
    const TS f2 = TS(0.5) * sf * sf - TS(0.25);
    const TS f3 = TS(-0.5) * sf * cf;
    pe = pe + TS(q[kPe2]) * f2 + TS(q[kPe3]) * f3;
    pinc = pinc + TS(q[kPi2]) * f2 + TS(q[kPi3]) * f3;
    pl = pl + TS(q[kPl2]) * f2 + TS(q[kPl3]) * f3 + TS(q[kPl4]) * sf;
    pgh = pgh + TS(q[kPgh2]) * f2 + TS(q[kPgh3]) * f3 + TS(q[kPgh4]) * sf;
    ph = ph + TS(q[kPh2]) * f2 + TS(q[kPh3]) * f3;
  }
  TS incp = incl + pinc;
  e = e + pe;
  TS si, ci;
  Trig<TS, TS>::sc(incp, &si, &ci);
  if (incp >= TS(0.2)) {
    ph = ph / si;
    argp = argp + pgh - ci * ph;
    node = node + ph;
    M = M + pl;
  } else {
    TS sn, cn;
    Trig<TS, TS>::sc(node, &sn, &cn);
    const TS alf = si * sn + (ph * cn + pinc * ci * sn);
    const TS bet = si * cn + (-ph * sn + pinc * ci * cn);
    const TS xls = M + argp + ci * node + (pl + pgh - pinc * node * si);
    const TS node_old = node;
    node = arctan2(alf, bet);
    if (vabs(node_old - node) > TS(kPi)) node = node < node_old ? node + twopi : node - twopi;
    M = M + pl;
    argp = xls - M - ci * node;
  }
  if (incp < TS(0)) {
    incp = -incp;
    node = node + TS(kPi);
    argp = argp - TS(kPi);
  }
  if (!(e >= TS(0) && e <= TS(1))) return 3;
  Trig<TS, TS>::sc(incp, &si, &ci);
  const TS cos2 = ci * ci;
  const TS j3oj2 = TS(g.j3oj2);
  const TS k2 = TS(g.k2);
  TS den = TS(1) + ci;
  if (vabs(den) <= TS(1.5e-12)) den = TS(1.5e-12);
  const TS c41 = TS(3) * cos2 - TS(1), x1 = TS(1) - cos2, x7 = TS(7) * cos2 - TS(1);
  const Incl<TS, TP> q{TP(c41), TP(x1), TP(x7), TP(ci), TP(si), TP(incp), TP(TS(-0.5) * j3oj2 * si),
                       TP(TS(-0.25) * j3oj2 * si * (TS(3) + TS(5) * ci) / den),
                       TP(TS(1.5) * k2 * c41), TP(TS(0.5) * k2 * x1), TP(k2 * x1), TP(TS(-0.25) * k2 * x7),
                       TP(TS(1.5) * k2 * ci), TP(TS(1.5) * k2 * ci * si)};
  return sgp4_tail<TS, TP>(g, TP(a_s), TP(e), M, argp, node, q, out);
}

// Returns the point's code (0, 1, 2, 3, 4 or 6).  r and v are written, and ok
// set, for codes 0 and 6 only.
//
// Secular part: sin M from sin/cos of the drag-free M by a small rotation
// (FP64; the float paths take the hardware sine of M), an identity up to
// rounding.  Deep-space satellites take deep_point (propagate_point branches
// before loading the constants).
template <class TS, class TP>
__device__ __forceinline__ uint32_t sgp4_point(const SatC<TS, TP>& c, const Grav& g, double t_abs, PointState<TP>& out) {
  using TR = Trig<TS, TP>;
  out.ok = false;
  const uint32_t scode = c.info & kInfoCodeMask;
  if (scode) return scode;

  // Secular gravity (secular type).
  const TS t = TS(t_abs - c.epoch_min);
  const TP tp = TP(t);
  const TS t2 = t * t;
  const TS Mdf = lin(c.M0, c.Mdot, t);
  const TS argpdf = lin(c.argp0, c.argpdot, t);
  TS node = lin(c.node0, c.nodedot, t) + c.nodecf * t2;
  TP a, e_s;
  TS M = Mdf, argp = argpdf;
  if constexpr (sizeof(TP) == 4) {
    // Float paths: 1 - A, the eccentricity decrement and the drag changes of
    // M and argp in float; the mean-anomaly polynomial L_d / t^2 (multiplied
    // by n0'' t^2, an angle of up to radians) in the secular type; all
    // polynomials in Horner form.
    TP dA = c.pC1 * tp;
    TP Ed = c.pbC4 * tp;
    TS Ld = c.t2cof;
    if (!(c.info & kInfoIsimp)) {
      TP sM, cM;
      TR::sc_damped(Mdf, &sM, &cM);
      const TP x = TP(1) + c.eta * cM;
      const TP dMa = vfma(c.pArgpcof, tp, c.pMcof * (x * x * x - c.dM0));
      M = Mdf + TS(dMa);
      argp = argpdf - TS(dMa);
      dA = tp * vfma(tp, vfma(tp, vfma(tp, c.pD4, c.pD3), c.pD2), c.pC1);
      // one hardware sine of M costs less than the rotation
      TR::sc_damped(M, &sM, &cM);
      Ed = vfma(c.pbC5, sM - c.sinM0, Ed);
      Ld = vfma(vfma(lin(c.t4cof, c.t5cof, t), t, c.t3cof), t, c.t2cof);
    }
    // a = a0'' A^2 = a0'' + a0'' (1 - A) ((1 - A) - 2)
    a = vfma(c.pA0pp, dA * (dA - TP(2)), c.pA0pp);
    e_s = c.pE0 - Ed;
    if (!(e_s >= TP(-0.001) && e_s < TP(1))) return 1;
    M = M + c.n0pp * (Ld * t2);
  } else {
    // FP64: sin M from sin/cos of the drag-free M by a small rotation
    TS A = TS(1) - c.C1 * t;
    TS Ed = c.bC4 * t;
    TS Ld = c.t2cof * t2;
    if (!(c.info & kInfoIsimp)) {
      TP sM, cM;
      TR::sc_damped(Mdf, &sM, &cM);
      const TP x = TP(1) + c.eta * cM;
      const TS dM = c.Mcof * TS(x * x * x - c.dM0);
      const TS dMa = c.argpcof * t + dM;
      M = Mdf + dMa;
      argp = argpdf - dMa;
      const TS t3 = t2 * t, t4 = t3 * t;
      A = A - c.D2 * t2 - c.D3 * t3 - c.D4 * t4;
      if (vabs(dMa) > TS(kRotMax)) TR::sc_damped(M, &sM, &cM);
      else rotate_small(&sM, &cM, TP(dMa));
      Ed = Ed + c.bC5 * TS(sM - c.sinM0);
      Ld = Ld + c.t3cof * t3 + t4 * lin(c.t4cof, c.t5cof, t);
    }
    a = TP(c.a0pp * A * A);
    e_s = TP(c.e0 - Ed);
    if (!(e_s >= TP(-0.001) && e_s < TP(1))) return 1;
    M = M + c.n0pp * Ld;
  }
  // Angles stay unreduced: every one of them only enters through sin/cos,
  // whose own reduction handles any size met here.

  // Eccentricity floor 1e-6.  e_s is not NaN here, so the maximum is the
  // floor: one instruction in float instead of a compare and two selects.
  const TP e = vmax(e_s, TP(1.0e-6));
  const Incl<TS, TP> q{c.c41, c.x1, c.x7, c.cosi, c.sini, c.i0, c.aycof, c.Lcof,
                       c.spA1, c.spX1h, c.spX1k, c.spX7q, c.spCN, c.spCI};
  return sgp4_tail<TS, TP>(g, a, e, M, argp, node, q, out);
}

// The satellite's info word alone (through the same view as its constants).
template <bool kVec>
__device__ __forceinline__ uint32_t load_info(const RecordView& rv, int64_t i) {
  if (kVec) return lane_slot(rv.slots + i)->info;
  return ((CSlot)(rv.slots + i))->info;
}

// Point of satellite i at t_abs: near-Earth, or the deep-space path.
//
// When the record holds no deep-space satellite (record_has_deep: two header
// words every wavefront shares) the constants and the info word load together
// and go to the near-Earth terms; otherwise the info word comes first and the
// branch precedes any other load (so the deep-space terms do not hold the
// near-Earth constants).  kDeep = false: an instantiation without the
// deep-space terms at all, for a ragged plan whose record held none when the
// plan was made; a deep-space satellite met anyway (the record re-initialised
// under the plan) gets code 7 and no state.
template <class TS, class TP, bool kVec, bool kDeep = true>
__device__ __forceinline__ uint32_t propagate_point(const RecordView& rv, int64_t i, const Grav& g, double t_abs,
                                                    PointState<TP>& out) {
  if (!kDeep || !record_has_deep(rv)) {
    const SatC<TS, TP> c = load_sat<TS, TP, kVec>(rv, i);
    if (c.info & kInfoDeep) {
      out.ok = false;
      return 7u;
    }
    return sgp4_point<TS, TP>(c, g, t_abs, out);
  }
  if (load_info<kVec>(rv, i) & kInfoDeep) {
    const SatC<TS, TP> c = load_sat<TS, TP, kVec>(rv, i);
    return deep_point<TS, TP>(c, g, t_abs, out);
  }
  const SatC<TS, TP> c = load_sat<TS, TP, kVec>(rv, i);
  return sgp4_point<TS, TP>(c, g, t_abs, out);
}

}  // namespace sgp4mi

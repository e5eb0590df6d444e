// Initialisation kernel: mean elements -> per-satellite constant record.
//
// One lane per satellite, double precision.  Computes the near-Earth SGP4
// initialisation of the published model the paper re-implements (section 2.1:
// Hoots & Roehrich 1980 / Hoots et al. 2004 / Vallado et al. 2006, WGS72):
// recovery of the original mean motion and semi-major axis from the element
// set's Kozai mean motion, the perigee-dependent atmospheric parameters, the
// power-law drag coefficients C1..C5 and D2..D4, the J2/J2^2/J4 secular rates
// and the J3 long-period coefficients.  The satellite-level validity checks
// (eccentricity at epoch, recovered mean motion, 225-minute deep-space
// boundary of section 6) are resolved here, once per satellite, so the
// per-point kernels only read a code.
#include "sgp4mi_common.h"

namespace sgp4mi {

struct InitArgs {
  int64_t n, npad;
  const double* elem;   // [8][n]
  double* hdr;
  Slot* slots;
  uint8_t* user_flags;  // nullable
  double mu, radius, j2, j3, j4;
};

__global__ void __launch_bounds__(256) init_kernel(InitArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const double ke = 60.0 / sqrt(a.radius * a.radius * a.radius / a.mu);
  const double j3oj2 = (a.j3 == 0.0) ? 0.0 : a.j3 / a.j2;
  if (i == 0) {
    double* h = a.hdr;
    h[kHMagic] = kMagic;
    h[kHN] = double(a.n);
    h[kHNpad] = double(a.npad);
    h[kHKe] = ke;
    h[kHRadius] = a.radius;
    h[kHVkms] = a.radius * ke / 60.0;
    h[kHK2] = 0.5 * a.j2;
    h[kHJ2] = a.j2;
    h[kHJ3oJ2] = j3oj2;
    h[kHJ4] = a.j4;
    h[kHMu] = a.mu;
  }
  if (i >= a.n) return;
  const int64_t n = a.n;
  const double no_kozai = a.elem[0 * n + i];
  const double ecco = a.elem[1 * n + i];
  const double inclo = a.elem[2 * n + i];
  const double nodeo = a.elem[3 * n + i];
  const double argpo = a.elem[4 * n + i];
  const double mo = a.elem[5 * n + i];
  const double bstar = a.elem[6 * n + i];
  const double epoch = a.elem[7 * n + i];
  const double R = a.radius, J2 = a.j2, J4 = a.j4;

  double sin_i, cos_i;
  sincos(inclo, &sin_i, &cos_i);
  const double c2 = cos_i * cos_i;
  const double omeosq = 1.0 - ecco * ecco;  // beta0^2
  const double rteosq = sqrt(omeosq);        // beta0
  const double con41 = 3.0 * c2 - 1.0;
  const double x1mth2 = 1.0 - c2;
  const double x7thm1 = 7.0 * c2 - 1.0;

  // Original mean motion: invert the Kozai definition with the second-order
  // correction of the published model.
  const double ak = cbrt(ke / no_kozai);
  const double a1 = ak * ak;
  const double d1 = 0.75 * J2 * con41 / (rteosq * omeosq);
  const double del1 = d1 / (a1 * a1);
  const double adel = a1 * (1.0 - del1 * (1.0 / 3.0 + del1 * (1.0 + (134.0 / 81.0) * del1)));
  const double del0 = d1 / (adel * adel);
  const double nbar = no_kozai / (1.0 + del0);
  const double ab = cbrt(ke / nbar);
  const double abar = ab * ab;

  // Perigee height -> density parameter s and (q0 - s)^4.
  const double perigee_er = abar * (1.0 - ecco);
  const double perigee_km = (perigee_er - 1.0) * R;
  double sfour = 1.0 + 78.0 / R;
  double qoms = (120.0 - 78.0) / R;
  if (perigee_km < 156.0) {
    double s_km = (perigee_km < 98.0) ? 20.0 : perigee_km - 78.0;
    qoms = (120.0 - s_km) / R;
    sfour = 1.0 + s_km / R;
  }
  const double qoms2 = qoms * qoms;
  const double qoms24 = qoms2 * qoms2;

  const bool isimp = perigee_er < 1.0 + 220.0 / R;
  uint32_t code = 0;
  if (!(ecco >= 0.0 && ecco < 1.0)) code = 1;
  else if (!(nbar > 0.0)) code = 2;
  else if (kTwoPi / nbar >= 225.0) code = 7;

  // Power-law drag coefficients.
  const double tsi = 1.0 / (abar - sfour);
  const double eta = abar * ecco * tsi;
  const double etasq = eta * eta;
  const double eeta = ecco * eta;
  const double psisq = fabs(1.0 - etasq);
  const double tsi2 = tsi * tsi;
  const double coef = qoms24 * tsi2 * tsi2;
  const double coef1 = coef / (psisq * psisq * psisq * sqrt(psisq));
  const double cc2 = coef1 * nbar *
                     (abar * (1.0 + 1.5 * etasq + eeta * (4.0 + etasq)) +
                      0.375 * J2 * tsi / psisq * con41 * (8.0 + 3.0 * etasq * (8.0 + etasq)));
  const double cc1 = bstar * cc2;
  const double cc3 = (ecco > 1.0e-4) ? -2.0 * coef * tsi * j3oj2 * nbar * sin_i / ecco : 0.0;
  double sin_2w, cos_2w;
  sincos(2.0 * argpo, &sin_2w, &cos_2w);
  const double cc4 = 2.0 * nbar * coef1 * abar * omeosq *
                     (eta * (2.0 + 0.5 * etasq) + ecco * (0.5 + 2.0 * etasq) -
                      J2 * tsi / (abar * psisq) *
                          (-3.0 * con41 * (1.0 - 2.0 * eeta + etasq * (1.5 - 0.5 * eeta)) +
                           0.75 * x1mth2 * (2.0 * etasq - eeta * (1.0 + etasq)) * cos_2w));
  const double cc5 = 2.0 * coef1 * abar * omeosq * (1.0 + 2.75 * (etasq + eeta) + eeta * etasq);

  // Secular rates.
  const double pinv = 1.0 / (abar * omeosq);
  const double pinvsq = pinv * pinv;
  const double c4 = c2 * c2;
  const double temp1 = 1.5 * J2 * pinvsq * nbar;
  const double temp2 = 0.5 * temp1 * J2 * pinvsq;
  const double temp3 = -0.46875 * J4 * pinvsq * pinvsq * nbar;
  const double mdot = nbar + 0.5 * temp1 * rteosq * con41 + 0.0625 * temp2 * rteosq * (13.0 - 78.0 * c2 + 137.0 * c4);
  const double argpdot = -0.5 * temp1 * (1.0 - 5.0 * c2) + 0.0625 * temp2 * (7.0 - 114.0 * c2 + 395.0 * c4) +
                         temp3 * (3.0 - 36.0 * c2 + 49.0 * c4);
  const double xhdot1 = -temp1 * cos_i;
  const double nodedot = xhdot1 + (0.5 * temp2 * (4.0 - 19.0 * c2) + 2.0 * temp3 * (3.0 - 7.0 * c2)) * cos_i;

  double sin_m0, cos_m0;
  sincos(mo, &sin_m0, &cos_m0);
  double argpcof = bstar * cc3 * cos(argpo);
  double xmcof = (ecco > 1.0e-4) ? -(2.0 / 3.0) * coef * bstar / eeta : 0.0;
  const double nodecf = 3.5 * omeosq * xhdot1 * cc1;
  const double t2cof = 1.5 * cc1;
  double den = 1.0 + cos_i;
  if (fabs(den) <= 1.5e-12) den = 1.5e-12;
  const double xlcof = -0.25 * j3oj2 * sin_i * (3.0 + 5.0 * cos_i) / den;
  const double aycof = -0.5 * j3oj2 * sin_i;
  const double dm = 1.0 + eta * cos_m0;
  const double delmo = dm * dm * dm;

  double d2 = 0, d3 = 0, d4 = 0, t3cof = 0, t4cof = 0, t5cof = 0, bc5 = bstar * cc5;
  if (!isimp) {
    const double cc1sq = cc1 * cc1;
    d2 = 4.0 * abar * tsi * cc1sq;
    const double tmp = d2 * tsi * cc1 / 3.0;
    d3 = (17.0 * abar + sfour) * tmp;
    d4 = 0.5 * tmp * abar * tsi * (221.0 * abar + 31.0 * sfour) * cc1;
    t3cof = d2 + 2.0 * cc1sq;
    t4cof = 0.25 * (3.0 * d3 + cc1 * (12.0 * d2 + 10.0 * cc1sq));
    t5cof = 0.2 * (3.0 * d4 + 12.0 * cc1 * d3 + 6.0 * d2 * d2 + 15.0 * cc1sq * (2.0 * d2 + cc1sq));
  } else {
    // The simplified model applies none of these; zeroing them makes the
    // general per-point expression reduce exactly to the simplified one.
    argpcof = 0.0;
    xmcof = 0.0;
    bc5 = 0.0;
  }

  double rec[kNRec];
  rec[kM0] = mo; rec[kMdot] = mdot; rec[kArgp0] = argpo; rec[kArgpdot] = argpdot;
  rec[kNode0] = nodeo; rec[kNodedot] = nodedot; rec[kNodecf] = nodecf; rec[kC1] = cc1;
  rec[kBC4] = bstar * cc4; rec[kT2cof] = t2cof; rec[kArgpcof] = argpcof; rec[kEta] = eta;
  rec[kMcof] = xmcof; rec[kDM0] = delmo; rec[kD2] = d2; rec[kD3] = d3; rec[kD4] = d4;
  rec[kBC5] = bc5; rec[kSinM0] = sin_m0; rec[kT3cof] = t3cof; rec[kT4cof] = t4cof; rec[kT5cof] = t5cof;
  rec[kN0pp] = nbar; rec[kA0pp] = abar; rec[kE0] = ecco; rec[kAycof] = aycof; rec[kLcof] = xlcof;
  rec[kC41] = con41; rec[kX1] = x1mth2; rec[kX7] = x7thm1; rec[kCosi] = cos_i; rec[kSini] = sin_i;
  rec[kI0] = inclo; rec[kEpochMin] = 1440.0 * epoch;
  Slot* slot = a.slots + i;
#pragma unroll
  for (int k = 0; k < kNRec; ++k) {
    slot->d[k] = rec[k];
    slot->f[k] = float(rec[k]);
  }
  slot->info = code | (isimp ? kInfoIsimp : 0u);
  if (a.user_flags) {
    uint8_t f = 0;
    if (code == 7) f |= 1;
    if (isimp) f |= 2;
    if (code == 1 || code == 2) f |= 4;
    a.user_flags[i] = f;
  }
}

hipError_t launch_init(const double g[5], int64_t n, const double* elem, void* consts, uint8_t* user_flags,
                       hipStream_t s) {
  InitArgs a;
  a.n = n;
  a.npad = npad_of(n);
  a.elem = elem;
  char* b = static_cast<char*>(consts);
  a.hdr = reinterpret_cast<double*>(b);
  a.slots = reinterpret_cast<Slot*>(b + kHCount * 8);
  a.user_flags = user_flags;
  a.mu = g[0]; a.radius = g[1]; a.j2 = g[2]; a.j3 = g[3]; a.j4 = g[4];
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(init_kernel, dim3(unsigned(blocks > 0 ? blocks : 1)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace sgp4mi

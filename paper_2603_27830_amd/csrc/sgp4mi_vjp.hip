// Vector-Jacobian product of the dense propagation with respect to the seven
// differentiated elements (paper section 5: gradients of the state with
// respect to the initial orbital elements, including B*).
//
// One workgroup per satellite.  Each lane recomputes the forward pass of its
// points (nothing from the forward launch is stored), then runs the reverse
// sweep of the per-point steps by hand, giving the adjoint of every
// per-satellite constant in double.  Kepler's equation is differentiated
// through the implicit-function theorem at its root.  Each lane accumulates
// the adjoints of its points; the workgroup then sums them in a fixed order
// (wavefront butterfly, then the wavefronts in index order: no atomics, so
// results repeat bit for bit), and seven lanes push the sums through the
// initialisation by forward-mode duals, one element each:
// g_m = sum_k cbar_k * d c_k / d theta_m.
#include "sgp4mi_initcore.h"
#include "sgp4mi_point.h"

namespace sgp4mi {

constexpr int kVjpBlock = 256;
// Workgroups per compute unit the register allocation must allow: two (two
// wavefronts per SIMD) in FP64, whose reverse sweep otherwise spills past 256
// registers and runs one wavefront per SIMD; three in the mixed path.
template <class TP> constexpr int kVjpBlocksPerCU = sizeof(TP) == 8 ? 2 : 3;

template <class TS, class TP>
__device__ __forceinline__ uint32_t point_vjp(const SatC<TS, TP>& c, const Grav& g, double t_abs, const TP gr[3],
                                          const TP gv[3], double* cb) {
  using TR = Trig<TS, TP>;
  if (c.info & kInfoCodeMask) return c.info & kInfoCodeMask;
  if (c.info & kInfoDeep) return 7;  // deep space: not differentiated
  const bool simp = (c.info & kInfoIsimp) != 0;

  // ---------------------------------------------------------- forward --
  // The forward kernel's formulation (reciprocals, small-angle rotations,
  // the argument of latitude kept as a (sin, cos) pair), keeping what the
  // reverse sweep needs.
  const TS t = TS(t_abs - c.epoch_min);
  const TS t2 = t * t, t3 = t2 * t, t4 = t3 * t;
  const TS Mdf = c.M0 + c.Mdot * t;
  const TS argpdf = c.argp0 + c.argpdot * t;
  const TS node = c.node0 + c.nodedot * t + c.nodecf * t2;
  TS A = TS(1) - c.C1 * t;
  TS Ed = c.bC4 * t;
  TS Ld = c.t2cof * t2;
  TS M = Mdf, argp = argpdf;
  TP sMdf = TP(0), cMdf = TP(1), x = TP(1), sM = TP(0), cM = TP(1);
  if (!simp) {
    TR::sc_damped(Mdf, &sMdf, &cMdf);
    x = TP(1) + c.eta * cMdf;
    const TS dM = c.Mcof * TS(x * x * x - c.dM0);
    const TS dMa = c.argpcof * t + dM;
    M = Mdf + dMa;
    argp = argpdf - dMa;
    A = A - c.D2 * t2 - c.D3 * t3 - c.D4 * t4;
    sM = sMdf;
    cM = cMdf;
    // As the forward kernel: float paths take the hardware sine and cosine of M.
    if (sizeof(TP) == 4 || vabs(dMa) > TS(kRotMax)) TR::sc_damped(M, &sM, &cM);
    else rotate_small(&sM, &cM, TP(dMa));
    Ed = Ed + c.bC5 * TS(sM - c.sinM0);
    Ld = Ld + c.t3cof * t3 + t4 * (c.t4cof + t * c.t5cof);
  }
  const TS a_s = c.a0pp * A * A;
  TS e_s = c.e0 - Ed;
  if (!(e_s >= TS(-0.001) && e_s < TS(1))) return 1;
  const bool clamped = e_s < TS(1.0e-6);
  if (clamped) e_s = TS(1.0e-6);
  const TP a = TP(a_s), e = TP(e_s);
  TP sw, cw;
  TR::sc_damped(argp, &sw, &cw);
  const TP axn = e * cw;
  const TP q = a * (TP(1) - e * e);
  const TP tau = rcp(q);
  const TP ayn = e * sw + tau * c.aycof;
  // U = L_T - node with L = M + n0 Ld + argp + node
  const TS U = M + c.n0pp * Ld + argp + TS(tau * c.Lcof * axn);
  TP sp, cp;
  TR::sc(U, &sp, &cp);
  {
    TP dpsi = TP(0);
    const TP eb = vabs(axn) + vabs(ayn);
    const TP quad = eb < TP(0.5) ? eb : TP(1.0e30);
    for (int k = 0; k < 10; ++k) {
      TP step = (axn * sp - ayn * cp - dpsi) * rcp(TP(1) - axn * cp - ayn * sp);
      step = clamp_step(step);
      dpsi = dpsi + step;
      if (vabs(step) <= TP(kRotMax)) rotate_small(&sp, &cp, step);
      else TR::sc(U + TS(dpsi), &sp, &cp);
      const TP as = vabs(step);
      if (__all(as < kepler_tol<TP>() || quad * as * as < kepler_tol<TP>())) break;
    }
  }
  const TP D = TP(1) - axn * cp - ayn * sp;
  const TP ecE = axn * cp + ayn * sp;
  const TP esE = axn * sp - ayn * cp;
  const TP eL2 = axn * axn + ayn * ayn;
  const TP pL = a * (TP(1) - eL2);
  if (!(pL >= TP(0))) return 4;
  const TP rl = a * (TP(1) - ecE);
  const TP irl = rcp(rl);
  const TP ra = rsq(a);
  const TP sqa = a * ra;
  const TP rdotl = sqa * esE * irl;
  const TP betal = sq_root(TP(1) - eL2);
  const TP sqp = sqa * betal;  // sqrt(pL)
  const TP rvdotl = sqp * irl;
  const TP opb = TP(1) + betal;
  const TP iopb = rcp(opb);
  const TP w = esE * iopb;
  const TP ar = a * irl;
  const TP f1 = sp - ayn - axn * w;
  const TP f2 = cp - axn + ayn * w;
  const TP sinu = ar * f1, cosu = ar * f2;
  const TP nu2 = sinu * sinu + cosu * cosu;
  const TP sin2u = TP(2) * sinu * cosu;
  const TP cos2u = TP(1) - TP(2) * sinu * sinu;
  const TP ipl = rcp(pL);
  const TP k2g = grav_k2<TP>(g);
  const TP k1 = k2g * ipl;
  const TP k2 = k1 * ipl;
  const TP nk = ra * ra * ra;  // a^-3/2
  const TP g1 = c.x1 * cos2u + TP(1.5) * c.c41;
  const TP mrt = rl * (TP(1) - TP(1.5) * k2 * betal * c.c41) + TP(0.5) * k1 * c.x1 * cos2u;
  const TP du = TP(-0.25) * k2 * c.x7 * sin2u;
  const TP dnode = TP(1.5) * k2 * c.cosi * sin2u;
  const TP dinc = TP(1.5) * k2 * c.cosi * c.sini * cos2u;
  const TP mvt = rdotl - nk * k1 * c.x1 * sin2u;
  const TP rvdot = rvdotl + nk * k1 * g1;
  TP ssu, csu, snod, cnod, sinc = c.sini, cinc = c.cosi;
  if (vabs(du) <= TP(kRotMax)) {
    const TP h = rsq(nu2);
    ssu = sinu * h;
    csu = cosu * h;
    rotate_small(&ssu, &csu, du);
  } else {
    TR::sc(TS(arctan2(sinu, cosu) + du), &ssu, &csu);
  }
  if (vabs(dinc) <= TP(kRotMax)) rotate_small(&sinc, &cinc, dinc);
  else TR::sc(TS(c.i0 + dinc), &sinc, &cinc);
  TR::sc(node + TS(dnode), &snod, &cnod);
  const TP xmx = -snod * cinc, xmy = cnod * cinc;
  const TP ux = xmx * ssu + cnod * csu, uy = xmy * ssu + snod * csu, uz = sinc * ssu;
  const TP vx = xmx * csu - cnod * ssu, vy = xmy * csu - snod * ssu, vz = sinc * csu;

  // ---------------------------------------------------------- reverse --
  const TP R = grav_radius<TP>(g), vk = grav_vkms<TP>(g);
  const TP mrt_b = R * (gr[0] * ux + gr[1] * uy + gr[2] * uz);
  const TP mvt_b = vk * (gv[0] * ux + gv[1] * uy + gv[2] * uz);
  const TP rvdot_b = vk * (gv[0] * vx + gv[1] * vy + gv[2] * vz);
  const TP ux_b = R * mrt * gr[0] + vk * mvt * gv[0];
  const TP uy_b = R * mrt * gr[1] + vk * mvt * gv[1];
  const TP uz_b = R * mrt * gr[2] + vk * mvt * gv[2];
  const TP vx_b = vk * rvdot * gv[0], vy_b = vk * rvdot * gv[1], vz_b = vk * rvdot * gv[2];
  const TP xmx_b = ux_b * ssu + vx_b * csu;
  const TP xmy_b = uy_b * ssu + vy_b * csu;
  TP cnod_b = ux_b * csu - vx_b * ssu + xmy_b * cinc;
  TP snod_b = uy_b * csu - vy_b * ssu - xmx_b * cinc;
  const TP sinc_b = uz_b * ssu + vz_b * csu;
  const TP cinc_b = -xmx_b * snod + xmy_b * cnod;
  const TP ssu_b = ux_b * xmx + uy_b * xmy + uz_b * sinc - vx_b * cnod - vy_b * snod;
  const TP csu_b = ux_b * cnod + uy_b * snod + vx_b * xmx + vy_b * xmy + vz_b * sinc;
  const TP xinc_b = sinc_b * cinc - cinc_b * sinc;
  const TP xnode_b = snod_b * cnod - cnod_b * snod;
  const TP su_b = ssu_b * csu - csu_b * ssu;

  // short-period periodics
  const TP nk_b = rvdot_b * k1 * g1 - mvt_b * k1 * c.x1 * sin2u;
  TP k1_b = rvdot_b * nk * g1 - mvt_b * nk * c.x1 * sin2u;
  TP x1_b = rvdot_b * nk * k1 * cos2u - mvt_b * nk * k1 * sin2u;
  TP cos2u_b = rvdot_b * nk * k1 * c.x1;
  TP c41_b = rvdot_b * nk * k1 * TP(1.5);
  const TP rdotl_b = mvt_b, rvdotl_b = rvdot_b;
  TP sin2u_b = -mvt_b * nk * k1 * c.x1;
  const TP i0_b = xinc_b;
  TP k2_b = xinc_b * TP(1.5) * c.cosi * c.sini * cos2u;
  TP cosi_b = xinc_b * TP(1.5) * k2 * c.sini * cos2u;
  const TP sini_b = xinc_b * TP(1.5) * k2 * c.cosi * cos2u;
  cos2u_b += xinc_b * TP(1.5) * k2 * c.cosi * c.sini;
  k2_b += xnode_b * TP(1.5) * c.cosi * sin2u;
  cosi_b += xnode_b * TP(1.5) * k2 * sin2u;
  sin2u_b += xnode_b * TP(1.5) * k2 * c.cosi;
  const TP u_b = su_b;
  k2_b -= su_b * TP(0.25) * c.x7 * sin2u;
  const TP x7_b = -su_b * TP(0.25) * k2 * sin2u;
  sin2u_b -= su_b * TP(0.25) * k2 * c.x7;
  TP rl_b = mrt_b * (TP(1) - TP(1.5) * k2 * betal * c.c41);
  k2_b -= mrt_b * rl * TP(1.5) * betal * c.c41;
  TP betal_b = -mrt_b * rl * TP(1.5) * k2 * c.c41;
  c41_b -= mrt_b * rl * TP(1.5) * k2 * betal;
  k1_b += mrt_b * TP(0.5) * c.x1 * cos2u;
  x1_b += mrt_b * TP(0.5) * k1 * cos2u;
  cos2u_b += mrt_b * TP(0.5) * k1 * c.x1;
  TP a_b = nk_b * TP(-1.5) * nk * ra * ra;
  k1_b += k2_b * ipl;
  const TP ipl_b = k2_b * k1 + k1_b * k2g;
  TP pL_b = -ipl_b * ipl * ipl;

  // short-period preliminaries
  const TP inu2 = rcp(nu2);
  const TP sinu_b = TP(-4) * sinu * cos2u_b + TP(2) * cosu * sin2u_b + u_b * cosu * inu2;
  const TP cosu_b = TP(2) * sinu * sin2u_b - u_b * sinu * inu2;
  const TP ar_b = sinu_b * f1 + cosu_b * f2;
  TP sp_b = sinu_b * ar, cp_b = cosu_b * ar;
  TP ayn_b = -sinu_b * ar + cosu_b * ar * w;
  TP axn_b = -sinu_b * ar * w - cosu_b * ar;
  const TP w_b = -sinu_b * ar * axn + cosu_b * ar * ayn;
  a_b += ar_b * irl;
  rl_b -= ar_b * ar * irl;
  TP esE_b = w_b * iopb;
  betal_b -= w_b * w * iopb;
  TP eL2_b = -betal_b * TP(0.5) * rcp(betal);
  pL_b += rvdotl_b * TP(0.5) * rcp(sqp) * irl;
  rl_b -= rvdotl_b * rvdotl * irl;
  a_b += rdotl_b * TP(0.5) * rdotl * ra * ra;
  esE_b += rdotl_b * sqa * irl;
  rl_b -= rdotl_b * rdotl * irl;
  a_b += rl_b * (TP(1) - ecE);
  const TP ecE_b = -rl_b * a;
  a_b += pL_b * (TP(1) - eL2);
  eL2_b -= pL_b * a;
  axn_b += TP(2) * axn * eL2_b + esE_b * sp + ecE_b * cp;
  ayn_b += TP(2) * ayn * eL2_b - esE_b * cp + ecE_b * sp;
  sp_b += esE_b * axn + ecE_b * ayn;
  cp_b += -esE_b * ayn + ecE_b * axn;
  const TP psi_b = sp_b * cp - cp_b * sp;

  // Kepler's equation at its root: d psi = (dU + sin psi daxn - cos psi dayn) / D
  const TP pD = psi_b * rcp(D);
  const TS U_b = TS(pD);
  axn_b += pD * sp;
  ayn_b -= pD * cp;

  // long-period periodics
  TS node_b = TS(xnode_b) - U_b;
  const TS L_b = U_b;  // through LT
  const TP LTb = TP(U_b);
  TP tau_b = LTb * c.Lcof * axn + ayn_b * c.aycof;
  const TP Lcof_b = LTb * tau * axn;
  axn_b += LTb * tau * c.Lcof;
  TP e_b = ayn_b * sw;
  const TP sw_b = ayn_b * e;
  const TP aycof_b = ayn_b * tau;
  const TP q_b = -tau_b * tau * tau;
  a_b += q_b * (TP(1) - e * e);
  e_b -= q_b * TP(2) * a * e;
  e_b += axn_b * cw;
  const TP cw_b = axn_b * e;
  TS argp_b = TS(sw_b * cw - cw_b * sw) + L_b;
  node_b += L_b;
  TS M_b = L_b;
  const TS n0pp_b = L_b * Ld;
  const TS Ld_b = L_b * c.n0pp;

  // secular drag and gravity
  const TS es_b = clamped ? TS(0) : TS(e_b);
  const TS Ed_b = -es_b;
  const TS as_b = TS(a_b);
  const TS A_b = as_b * TS(2) * c.a0pp * A;
  TS Mdf_b, argpdf_b;
  cb[kE0] += double(es_b);
  cb[kA0pp] += double(as_b * A * A);
  cb[kN0pp] += double(n0pp_b);
  cb[kC1] += double(-A_b * t);
  cb[kBC4] += double(Ed_b * t);
  cb[kT2cof] += double(Ld_b * t2);
  if (!simp) {
    cb[kT3cof] += double(Ld_b * t3);
    cb[kT4cof] += double(Ld_b * t4);
    cb[kT5cof] += double(Ld_b * t4 * t);
    cb[kD2] += double(-A_b * t2);
    cb[kD3] += double(-A_b * t3);
    cb[kD4] += double(-A_b * t4);
    cb[kBC5] += double(Ed_b * TS(sM - c.sinM0));
    const TP sM_b = TP(Ed_b * c.bC5);
    cb[kSinM0] += double(-sM_b);
    M_b += TS(sM_b * cM);
    const TS dMa_b = M_b - argp_b;
    Mdf_b = M_b;
    argpdf_b = argp_b;
    cb[kArgpcof] += double(dMa_b * t);
    cb[kMcof] += double(dMa_b * TS(x * x * x - c.dM0));
    const TP x_b = TP(dMa_b * c.Mcof) * TP(3) * x * x;
    cb[kDM0] += double(-TP(dMa_b * c.Mcof));
    cb[kEta] += double(x_b * cMdf);
    Mdf_b += TS(-x_b * c.eta * sMdf);
  } else {
    Mdf_b = M_b;
    argpdf_b = argp_b;
  }
  cb[kM0] += double(Mdf_b);
  cb[kMdot] += double(Mdf_b * t);
  cb[kArgp0] += double(argpdf_b);
  cb[kArgpdot] += double(argpdf_b * t);
  cb[kNode0] += double(node_b);
  cb[kNodedot] += double(node_b * t);
  cb[kNodecf] += double(node_b * t2);
  cb[kAycof] += double(aycof_b);
  cb[kLcof] += double(Lcof_b);
  cb[kC41] += double(c41_b);
  cb[kX1] += double(x1_b);
  cb[kX7] += double(x7_b);
  cb[kCosi] += double(cosi_b);
  cb[kSini] += double(sini_b);
  cb[kI0] += double(i0_b);
  return mrt < TP(1) ? 6u : 0u;
}

// One workgroup's satellite i: its points p0 + j for j < cnt, at times tt[j],
// with cotangent rows of P entries (dense: p0 = i T, tt = t; CSR: p0 =
// offsets[i], tt = t + p0).
template <class TS, class TP>
__device__ __forceinline__ void vjp_sat(const RecordView& rv, int64_t n, const double* __restrict__ elem, int64_t i,
                                        int64_t p0, int64_t cnt, int64_t P, const double* __restrict__ tt,
                                        const TP* __restrict__ gr, const TP* __restrict__ gv,
                                        double* __restrict__ gelem) {
  constexpr int kWaves = kVjpBlock / 64;
  __shared__ double part[kWaves][kNRec];
  __shared__ double cbar[kNRec];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const SatC<TS, TP> c = load_sat<TS, TP, false>(rv, i);
  const Grav g = load_grav(rv);
  double acc[kNRec];
#pragma unroll
  for (int k = 0; k < kNRec; ++k) acc[k] = 0.0;
  const double* t = tt;
  for (int64_t j = threadIdx.x; j < cnt; j += kVjpBlock) {
    const int64_t p = p0 + j;
    const TP grp[3] = {gr[p], gr[P + p], gr[2 * P + p]};
    TP gvp[3] = {TP(0), TP(0), TP(0)};
    if (gv) {
      gvp[0] = gv[p];
      gvp[1] = gv[P + p];
      gvp[2] = gv[2 * P + p];
    }
    point_vjp<TS, TP>(c, g, t[j], grp, gvp, acc);
  }
  // fixed-order reduction: butterfly within the wavefront, then wavefronts in order
#pragma unroll
  for (int k = 0; k < kNRec; ++k) {
    double x = acc[k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) part[wave][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < kNRec) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += part[w][threadIdx.x];
    cbar[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int m = threadIdx.x;
    // deep-space satellites are not differentiated: NaN
    double out = (c.info & kInfoDeep) ? __builtin_nan("") : 0.0;
    if ((c.info & (kInfoCodeMask | kInfoDeep)) == 0) {
      Dual1 el[7];
      for (int k = 0; k < 7; ++k) el[k] = Dual1(elem[k * n + i], k == m ? 1.0 : 0.0);
      const double R = rv.hdr[kHRadius];
      GravIn gi{R, rv.hdr[kHJ2], rv.hdr[kHJ4], rv.hdr[kHKe], rv.hdr[kHJ3oJ2]};
      Dual1 rec[kNRec];
      uint32_t code;
      bool isimp, dsp;
      init_record<Dual1>(gi, el, rec, &code, &isimp, &dsp);
      for (int k = 0; k < kNRec; ++k)
        if (k != kEpochMin && cbar[k] != 0.0) out += cbar[k] * rec[k].d;
    }
    gelem[m * n + i] = out;
  }
}

template <class TS, class TP>
__global__ void __launch_bounds__(kVjpBlock, kVjpBlocksPerCU<TP>)
    vjp_kernel(RecordView rv, int64_t n, const double* __restrict__ elem, const double* __restrict__ t, int64_t T,
               const TP* __restrict__ gr, const TP* __restrict__ gv, double* __restrict__ gelem) {
  const int64_t i = blockIdx.x;
  vjp_sat<TS, TP>(rv, n, elem, i, i * T, T, n * T, t, gr, gv, gelem);
}

// CSR time lists: satellite i's points offsets[i] .. offsets[i+1]-1.  Each
// workgroup clamps its two offsets to [0, nnz] (and the end to at least the
// start), so malformed offsets never read outside t, gr or gv.
template <class TS, class TP>
__global__ void __launch_bounds__(kVjpBlock, kVjpBlocksPerCU<TP>)
    vjp_ragged_kernel(RecordView rv, int64_t n, const double* __restrict__ elem, const int64_t* __restrict__ offsets,
                      const double* __restrict__ t, int64_t nnz, const TP* __restrict__ gr,
                      const TP* __restrict__ gv, double* __restrict__ gelem) {
  const int64_t i = blockIdx.x;
  int64_t lo = offsets[i], hi = offsets[i + 1];
  lo = lo < 0 ? 0 : (lo > nnz ? nnz : lo);
  hi = hi < lo ? lo : (hi > nnz ? nnz : hi);
  vjp_sat<TS, TP>(rv, n, elem, i, lo, hi - lo, nnz, t + lo, gr, gv, gelem);
}

// Jacobian of the dense propagation (paper section 5: the state's sensitivity
// to the elements, the state-transition and covariance use):
// jac[(c * 7 + m) * P + p] = d state_c / d theta_m at point p, c over r_x, r_y,
// r_z, v_x, v_y, v_z and m over the seven differentiated elements; NaN where
// the point's code is 1, 2, 4 or 7.
//
// Forward mode: one workgroup per satellite; seven lanes first push the unit
// tangents of the elements through the initialisation (forward-mode duals)
// into the constants' sensitivities dc[m][k] = dc_k / dtheta_m (LDS).  Then
// every lane carries the seven tangents of each intermediate of its point
// through one pass of the forward kernel's formulation, beside the values:
// each step's tangent is its derivative applied to its inputs' tangents, and
// Kepler's equation is differentiated at its root (implicit-function theorem:
// dpsi = (dU + sin psi daxn - cos psi dayn) / (1 - axn cos psi - ayn sin psi)).
// The six state tangents are the point's Jacobian columns, stored as they
// come.  Secular tangents are double; periodic ones take the periodic type.

// Tangents of one intermediate in kN of the seven directions (elements kM0 ..
// kM0 + kN - 1): the directions are carried in groups, each group a pass of
// its own, so that the tangents fit the register file.
template <int kM0, int kN>
struct Dirs {
  static constexpr int m0 = kM0, n = kN;
};
template <class T, class D>
struct Tan7 {
  T d[D::n];
};

// Tangents of record constant k from the sensitivities in LDS.
template <class T, class D>
__device__ __forceinline__ Tan7<T, D> ctan(const double (*dc)[kNRec], int k) {
  Tan7<T, D> r;
#pragma unroll
  for (int m = 0; m < D::n; ++m) r.d[m] = T(dc[D::m0 + m][k]);
  return r;
}

// x' = a u' + b v' (and variants), elementwise over the seven directions.
template <class T, class D>
__device__ __forceinline__ Tan7<T, D> tlin(T a, const Tan7<T, D>& u) {
  Tan7<T, D> r;
#pragma unroll
  for (int m = 0; m < D::n; ++m) r.d[m] = a * u.d[m];
  return r;
}
template <class T, class D>
__device__ __forceinline__ Tan7<T, D> tlin(T a, const Tan7<T, D>& u, T b, const Tan7<T, D>& v) {
  Tan7<T, D> r;
#pragma unroll
  for (int m = 0; m < D::n; ++m) r.d[m] = fma(a, u.d[m], b * v.d[m]);
  return r;
}
template <class T, class D>
__device__ __forceinline__ Tan7<T, D> tlin(T a, const Tan7<T, D>& u, T b, const Tan7<T, D>& v, T c, const Tan7<T, D>& w) {
  Tan7<T, D> r;
#pragma unroll
  for (int m = 0; m < D::n; ++m) r.d[m] = fma(a, u.d[m], fma(b, v.d[m], c * w.d[m]));
  return r;
}
// acc += a u'
template <class T, class D>
__device__ __forceinline__ void tacc(Tan7<T, D>& acc, T a, const Tan7<T, D>& u) {
#pragma unroll
  for (int m = 0; m < D::n; ++m) acc.d[m] = fma(a, u.d[m], acc.d[m]);
}
template <class TO, class TI, class D>
__device__ __forceinline__ Tan7<TO, D> tcast(const Tan7<TI, D>& u) {
  Tan7<TO, D> r;
#pragma unroll
  for (int m = 0; m < D::n; ++m) r.d[m] = TO(u.d[m]);
  return r;
}

// One point: the state's seven tangents (jr[c], jv[c] for c = x, y, z), or the
// point's code when it carries no state (1, 2, 4, 7).
template <class TS, class TP, class D>
__device__ __forceinline__ uint32_t point_jvp(const SatC<TS, TP>& c, const Grav& g, double t_abs,
                                              const double (*dc)[kNRec], Tan7<TP, D> jr[3], Tan7<TP, D> jv[3]) {
  using TR = Trig<TS, TP>;
  if (c.info & kInfoCodeMask) return c.info & kInfoCodeMask;
  if (c.info & kInfoDeep) return 7;  // deep space: not differentiated
  const bool simp = (c.info & kInfoIsimp) != 0;

  // Secular gravity and drag (tangents in TS).
  const TS t = TS(t_abs - c.epoch_min);
  const TS t2 = t * t, t3 = t2 * t, t4 = t3 * t;
  const TS Mdf = c.M0 + c.Mdot * t;
  const TS argpdf = c.argp0 + c.argpdot * t;
  const TS node = c.node0 + c.nodedot * t + c.nodecf * t2;
  Tan7<TS, D> Mdf_t = tlin(TS(1), ctan<TS, D>(dc, kM0), t, ctan<TS, D>(dc, kMdot));
  Tan7<TS, D> argp_t = tlin(TS(1), ctan<TS, D>(dc, kArgp0), t, ctan<TS, D>(dc, kArgpdot));
  Tan7<TS, D> node_t = tlin(TS(1), ctan<TS, D>(dc, kNode0), t, ctan<TS, D>(dc, kNodedot), t2, ctan<TS, D>(dc, kNodecf));
  TS A = TS(1) - c.C1 * t;
  Tan7<TS, D> A_t = tlin(-t, ctan<TS, D>(dc, kC1));
  TS Ed = c.bC4 * t;
  Tan7<TS, D> Ed_t = tlin(t, ctan<TS, D>(dc, kBC4));
  TS Ld = c.t2cof * t2;
  Tan7<TS, D> Ld_t = tlin(t2, ctan<TS, D>(dc, kT2cof));
  TS M = Mdf, argp = argpdf;
  Tan7<TS, D> M_t = Mdf_t;
  if (!simp) {
    TP sMdf, cMdf;
    TR::sc_damped(Mdf, &sMdf, &cMdf);
    const TP x = TP(1) + c.eta * cMdf;
    // x' = eta' cos Mdf - eta sin Mdf Mdf'
    const Tan7<TS, D> x_t = tlin(TS(cMdf), ctan<TS, D>(dc, kEta), TS(-c.eta * sMdf), Mdf_t);
    const TS x3 = TS(x * x * x - c.dM0);
    const TS dM = c.Mcof * x3;
    // dMa = argpcof t + Mcof (x^3 - dM0)
    Tan7<TS, D> dMa_t = tlin(t, ctan<TS, D>(dc, kArgpcof), x3, ctan<TS, D>(dc, kMcof), TS(-c.Mcof), ctan<TS, D>(dc, kDM0));
    tacc(dMa_t, TS(c.Mcof * TS(TP(3) * x * x)), x_t);
    const TS dMa = c.argpcof * t + dM;
    M = Mdf + dMa;
    argp = argpdf - dMa;
#pragma unroll
    for (int m = 0; m < D::n; ++m) {
      M_t.d[m] += dMa_t.d[m];
      argp_t.d[m] -= dMa_t.d[m];
    }
    A = A - c.D2 * t2 - c.D3 * t3 - c.D4 * t4;
    tacc(A_t, -t2, ctan<TS, D>(dc, kD2));
    tacc(A_t, -t3, ctan<TS, D>(dc, kD3));
    tacc(A_t, -t4, ctan<TS, D>(dc, kD4));
    TP sM = sMdf, cM = cMdf;
    if (sizeof(TP) == 4 || vabs(dMa) > TS(kRotMax)) TR::sc_damped(M, &sM, &cM);
    else rotate_small(&sM, &cM, TP(dMa));
    // Ed += bC5 (sin M - sinM0)
    const TS dsM = TS(sM - c.sinM0);
    Ed = Ed + c.bC5 * dsM;
    tacc(Ed_t, dsM, ctan<TS, D>(dc, kBC5));
    tacc(Ed_t, TS(c.bC5 * TS(cM)), M_t);
    tacc(Ed_t, -c.bC5, ctan<TS, D>(dc, kSinM0));
    Ld = Ld + c.t3cof * t3 + t4 * (c.t4cof + t * c.t5cof);
    tacc(Ld_t, t3, ctan<TS, D>(dc, kT3cof));
    tacc(Ld_t, t4, ctan<TS, D>(dc, kT4cof));
    tacc(Ld_t, t4 * t, ctan<TS, D>(dc, kT5cof));
  }
  const TS a_s = c.a0pp * A * A;
  // a' = a0pp' A^2 + 2 a0pp A A'
  const Tan7<TS, D> as_t = tlin(A * A, ctan<TS, D>(dc, kA0pp), TS(2) * c.a0pp * A, A_t);
  TS e_s = c.e0 - Ed;
  if (!(e_s >= TS(-0.001) && e_s < TS(1))) return 1;
  Tan7<TS, D> es_t = tlin(TS(1), ctan<TS, D>(dc, kE0), TS(-1), Ed_t);
  // M + n0 Ld (the mean longitude's drag term)
  const TS Mn = M + c.n0pp * Ld;
  tacc(M_t, Ld, ctan<TS, D>(dc, kN0pp));
  tacc(M_t, c.n0pp, Ld_t);

  // Long-period periodics (TP from here).
  const TP a = TP(a_s);
  TP e = TP(e_s);
  if (e < TP(1.0e-6)) {
    e = TP(1.0e-6);
#pragma unroll
    for (int m = 0; m < D::n; ++m) es_t.d[m] = TS(0);
  }
  const Tan7<TP, D> a_t = tcast<TP, TS, D>(as_t), e_t = tcast<TP, TS, D>(es_t), w_t = tcast<TP, TS, D>(argp_t);
  TP sw, cw;
  TR::sc_damped(argp, &sw, &cw);
  const TP axn = e * cw;
  Tan7<TP, D> axn_t = tlin(cw, e_t, -e * sw, w_t);
  const TP q = a * (TP(1) - e * e);
  const TP tau = rcp(q);
  const TP ayn = e * sw + tau * c.aycof;
  // tau' = -tau^2 (a' (1 - e^2) - 2 a e e')
  const Tan7<TP, D> tau_t = tlin(-tau * tau * (TP(1) - e * e), a_t, TP(2) * tau * tau * a * e, e_t);
  Tan7<TP, D> ayn_t = tlin(sw, e_t, e * cw, w_t, c.aycof, tau_t);
  tacc(ayn_t, tau, ctan<TP, D>(dc, kAycof));
  const TP LT = tau * c.Lcof * axn;
  const TS U = Mn + argp + TS(LT);
  // U' = M' + argp' + (tau Lcof axn)'
  Tan7<TP, D> U_t = tlin(c.Lcof * axn, tau_t, tau * axn, ctan<TP, D>(dc, kLcof), tau * c.Lcof, axn_t);
#pragma unroll
  for (int m = 0; m < D::n; ++m) U_t.d[m] += TP(M_t.d[m] + argp_t.d[m]);

  // Kepler, as the forward kernel.
  TP sp, cp;
  TR::sc(U, &sp, &cp);
  {
    TP dpsi = TP(0);
    const TP eb = vabs(axn) + vabs(ayn);
    const TP quad = eb < TP(0.5) ? eb : TP(1.0e30);
    for (int k = 0; k < 10; ++k) {
      TP step = (axn * sp - ayn * cp - dpsi) * rcp(TP(1) - axn * cp - ayn * sp);
      step = clamp_step(step);
      dpsi = dpsi + step;
      if (vabs(step) <= TP(kRotMax)) rotate_small(&sp, &cp, step);
      else TR::sc(U + TS(dpsi), &sp, &cp);
      const TP as = vabs(step);
      if (__all(as < kepler_tol<TP>() || quad * as * as < kepler_tol<TP>())) break;
    }
  }
  const TP iD = rcp(TP(1) - axn * cp - ayn * sp);
  // psi' = (U' + sin psi axn' - cos psi ayn') / D; then (sin psi, cos psi)' = (cos, -sin) psi'
  const Tan7<TP, D> psi_t = tlin(iD, U_t, sp * iD, axn_t, -cp * iD, ayn_t);

  // Short-period preliminaries.
  const TP ecE = axn * cp + ayn * sp;
  const TP esE = axn * sp - ayn * cp;
  const TP eL2 = axn * axn + ayn * ayn;
  // ecE' = cp axn' + sp ayn' - esE psi'; esE' = sp axn' - cp ayn' + ecE psi'
  const Tan7<TP, D> ecE_t = tlin(cp, axn_t, sp, ayn_t, -esE, psi_t);
  const Tan7<TP, D> esE_t = tlin(sp, axn_t, -cp, ayn_t, ecE, psi_t);
  const Tan7<TP, D> eL2_t = tlin(TP(2) * axn, axn_t, TP(2) * ayn, ayn_t);
  const TP pL = a * (TP(1) - eL2);
  if (!(pL >= TP(0))) return 4;
  const Tan7<TP, D> pL_t = tlin(TP(1) - eL2, a_t, -a, eL2_t);
  const TP rl = a * (TP(1) - ecE);
  const Tan7<TP, D> rl_t = tlin(TP(1) - ecE, a_t, -a, ecE_t);
  const TP irl = rcp(rl);
  const TP ra = rsq(a);
  const TP sqa = a * ra;
  const TP ia = ra * ra;
  const TP rdotl = sqa * esE * irl;
  // rdotl' = rdotl (a'/(2a) + esE'/esE - rl'/rl), written without 1/esE
  const Tan7<TP, D> rdotl_t = tlin(TP(0.5) * rdotl * ia, a_t, sqa * irl, esE_t, -rdotl * irl, rl_t);
  const TP betal = sq_root(TP(1) - eL2);
  const TP ibetal = rcp(betal);
  const Tan7<TP, D> betal_t = tlin(TP(-0.5) * ibetal, eL2_t);
  const TP rvdotl = sqa * betal * irl;
  const Tan7<TP, D> rvdotl_t = tlin(TP(0.5) * rvdotl * ia, a_t, sqa * irl, betal_t, -rvdotl * irl, rl_t);
  const TP iopb = rcp(TP(1) + betal);
  const TP w = esE * iopb;
  const Tan7<TP, D> w_tan = tlin(iopb, esE_t, -w * iopb, betal_t);
  const TP ar = a * irl;
  const Tan7<TP, D> ar_t = tlin(irl, a_t, -ar * irl, rl_t);
  const TP f1 = sp - ayn - axn * w;
  const TP f2 = cp - axn + ayn * w;
  // f1' = cp psi' - ayn' - w axn' - axn w'; f2' = -sp psi' - axn' + w ayn' + ayn w'
  Tan7<TP, D> f1_t = tlin(cp, psi_t, -TP(1), ayn_t, -w, axn_t);
  tacc(f1_t, -axn, w_tan);
  Tan7<TP, D> f2_t = tlin(-sp, psi_t, -TP(1), axn_t, w, ayn_t);
  tacc(f2_t, ayn, w_tan);
  const TP sinu = ar * f1, cosu = ar * f2;
  const Tan7<TP, D> sinu_t = tlin(f1, ar_t, ar, f1_t);
  const Tan7<TP, D> cosu_t = tlin(f2, ar_t, ar, f2_t);
  const TP sin2u = TP(2) * sinu * cosu;
  const TP cos2u = TP(1) - TP(2) * sinu * sinu;
  const Tan7<TP, D> sin2u_t = tlin(TP(2) * cosu, sinu_t, TP(2) * sinu, cosu_t);
  const Tan7<TP, D> cos2u_t = tlin(TP(-4) * sinu, sinu_t);

  // Short-period periodics (J2).
  const TP ipl = rcp(pL);
  const TP k2g = grav_k2<TP>(g);
  const TP k1 = k2g * ipl;
  const TP k2 = k1 * ipl;
  const Tan7<TP, D> k1_t = tlin(-k1 * ipl, pL_t);
  const Tan7<TP, D> k2_t = tlin(TP(-2) * k2 * ipl, pL_t);
  const TP nk = ra * ra * ra;  // a^-3/2
  const Tan7<TP, D> nk_t = tlin(TP(-1.5) * nk * ia, a_t);
  const Tan7<TP, D> c41_t = ctan<TP, D>(dc, kC41), x1_t = ctan<TP, D>(dc, kX1);
  const TP c41h = TP(1.5) * c.c41;
  const TP bk = TP(1) - k2 * betal * c41h;
  const TP mrt = rl * bk + TP(0.5) * k1 * c.x1 * cos2u;
  // mrt' = rl' bk - 1.5 rl (k2' betal c41 + k2 betal' c41 + k2 betal c41') + 0.5 (k1' x1 cos2u + k1 x1' cos2u + k1 x1 cos2u')
  Tan7<TP, D> mrt_t = tlin(bk, rl_t, -rl * betal * c41h, k2_t, -rl * k2 * c41h, betal_t);
  tacc(mrt_t, TP(-1.5) * rl * k2 * betal, c41_t);
  tacc(mrt_t, TP(0.5) * c.x1 * cos2u, k1_t);
  tacc(mrt_t, TP(0.5) * k1 * cos2u, x1_t);
  tacc(mrt_t, TP(0.5) * k1 * c.x1, cos2u_t);
  const TP du = TP(-0.25) * k2 * c.x7 * sin2u;
  Tan7<TP, D> du_t = tlin(TP(-0.25) * c.x7 * sin2u, k2_t, TP(-0.25) * k2 * sin2u, ctan<TP, D>(dc, kX7),
                       TP(-0.25) * k2 * c.x7, sin2u_t);
  const TP dnode = TP(1.5) * k2 * c.cosi * sin2u;
  Tan7<TP, D> dnode_t = tlin(TP(1.5) * c.cosi * sin2u, k2_t, TP(1.5) * k2 * sin2u, ctan<TP, D>(dc, kCosi),
                          TP(1.5) * k2 * c.cosi, sin2u_t);
  const TP dinc = TP(1.5) * k2 * c.cosi * c.sini * cos2u;
  Tan7<TP, D> dinc_t = tlin(TP(1.5) * c.cosi * c.sini * cos2u, k2_t, TP(1.5) * k2 * c.sini * cos2u,
                         ctan<TP, D>(dc, kCosi), TP(1.5) * k2 * c.cosi * cos2u, ctan<TP, D>(dc, kSini));
  tacc(dinc_t, TP(1.5) * k2 * c.cosi * c.sini, cos2u_t);
  const TP kx = nk * k1 * c.x1;
  const TP mvt = rdotl - kx * sin2u;
  // mvt' = rdotl' - (nk k1 x1)' sin2u - nk k1 x1 sin2u'
  Tan7<TP, D> mvt_t = tlin(TP(1), rdotl_t, -k1 * c.x1 * sin2u, nk_t, -nk * c.x1 * sin2u, k1_t);
  tacc(mvt_t, -nk * k1 * sin2u, x1_t);
  tacc(mvt_t, -kx, sin2u_t);
  const TP g1 = c.x1 * cos2u + c41h;
  const TP rvdot = rvdotl + nk * k1 * g1;
  Tan7<TP, D> rvdot_t = tlin(TP(1), rvdotl_t, k1 * g1, nk_t, nk * g1, k1_t);
  tacc(rvdot_t, nk * k1 * cos2u, x1_t);
  tacc(rvdot_t, nk * k1 * c.x1, cos2u_t);
  tacc(rvdot_t, TP(1.5) * nk * k1, c41_t);

  // Orientation: u_k = u + du, i_k = i0 + dinc, node_k = node + dnode.
  const TP nu2 = sinu * sinu + cosu * cosu;
  const TP inu2 = rcp(nu2);
  TP ssu, csu;
  if (vabs(du) <= TP(kRotMax)) {
    const TP h = rsq(nu2);
    ssu = sinu * h;
    csu = cosu * h;
    rotate_small(&ssu, &csu, du);
  } else {
    TR::sc(TS(arctan2(sinu, cosu) + du), &ssu, &csu);
  }
  // u' = (cosu sinu' - sinu cosu') / |.|^2
  Tan7<TP, D> uk_t = tlin(cosu * inu2, sinu_t, -sinu * inu2, cosu_t);
#pragma unroll
  for (int m = 0; m < D::n; ++m) uk_t.d[m] += du_t.d[m];
  TP sinc = c.sini, cinc = c.cosi;
  if (vabs(dinc) <= TP(kRotMax)) rotate_small(&sinc, &cinc, dinc);
  else TR::sc(TS(c.i0 + dinc), &sinc, &cinc);
  Tan7<TP, D> ik_t = ctan<TP, D>(dc, kI0);
#pragma unroll
  for (int m = 0; m < D::n; ++m) ik_t.d[m] += dinc_t.d[m];
  TP snod, cnod;
  TR::sc(node + TS(dnode), &snod, &cnod);
  Tan7<TP, D> nodek_t = tcast<TP, TS, D>(node_t);
#pragma unroll
  for (int m = 0; m < D::n; ++m) nodek_t.d[m] += dnode_t.d[m];

  const TP xmx = -snod * cinc, xmy = cnod * cinc;
  const TP ux = xmx * ssu + cnod * csu, uy = xmy * ssu + snod * csu, uz = sinc * ssu;
  const TP vx = xmx * csu - cnod * ssu, vy = xmy * csu - snod * ssu, vz = sinc * csu;
  // d(unit vectors) = vx du_k... written per direction from the three angle tangents:
  //   d ux = (xmx csu - cnod ssu) uk' + (-cnod cinc ssu - snod csu) nodek' + (snod sinc ssu) ik'
  //   d uy = (xmy csu - snod ssu) uk' + (-snod cinc ssu + cnod csu) nodek' + (-cnod sinc ssu) ik'
  //   d uz = (sinc csu) uk' + (cinc ssu) ik'
  //   d vx = (-xmx ssu - cnod csu) uk' + (-cnod cinc csu + snod ssu) nodek' + (snod sinc csu) ik'
  //   d vy = (-xmy ssu - snod csu) uk' + (-snod cinc csu - cnod ssu) nodek' + (-cnod sinc csu) ik'
  //   d vz = (-sinc ssu) uk' + (cinc csu) ik'
  const TP R = grav_radius<TP>(g), vk = grav_vkms<TP>(g);
  const TP rr = R * mrt;
  const TP xn_u = -cnod * cinc * ssu - snod * csu, yn_u = -snod * cinc * ssu + cnod * csu;
  const TP xn_v = -cnod * cinc * csu + snod * ssu, yn_v = -snod * cinc * csu - cnod * ssu;
  const TP sss = sinc * ssu, ssc = sinc * csu;
#pragma unroll
  for (int m = 0; m < D::n; ++m) {
    const TP du_ = uk_t.d[m], dn = nodek_t.d[m], di = ik_t.d[m];
    const TP dux = vx * du_ + xn_u * dn + snod * sss * di;
    const TP duy = vy * du_ + yn_u * dn - cnod * sss * di;
    const TP duz = vz * du_ + cinc * ssu * di;
    const TP dvx = -ux * du_ + xn_v * dn + snod * ssc * di;
    const TP dvy = -uy * du_ + yn_v * dn - cnod * ssc * di;
    const TP dvz = -uz * du_ + cinc * csu * di;
    const TP dmrt = R * mrt_t.d[m];
    jr[0].d[m] = fma(dmrt, ux, rr * dux);
    jr[1].d[m] = fma(dmrt, uy, rr * duy);
    jr[2].d[m] = fma(dmrt, uz, rr * duz);
    const TP dmvt = mvt_t.d[m], drv = rvdot_t.d[m];
    jv[0].d[m] = vk * (dmvt * ux + mvt * dux + drv * vx + rvdot * dvx);
    jv[1].d[m] = vk * (dmvt * uy + mvt * duy + drv * vy + rvdot * dvy);
    jv[2].d[m] = vk * (dmvt * uz + mvt * duz + drv * vz + rvdot * dvz);
  }
  return mrt < TP(1) ? 6u : 0u;
}

// One group of directions for one point: tangents and their stores.
template <class TS, class TP, class D>
__device__ __forceinline__ void jacobian_pass(const SatC<TS, TP>& c, const Grav& g, double tj,
                                              const double (*dc)[kNRec], double* __restrict__ jac, int64_t P,
                                              int64_t p) {
  Tan7<TP, D> jr[3], jv[3];
  const uint32_t code = point_jvp<TS, TP, D>(c, g, tj, dc, jr, jv);
  const bool ok = code == 0 || code == 6;
  const double qnan = __builtin_nan("");
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int m = 0; m < D::n; ++m) {
      st_nt(jac + (q * 7 + D::m0 + m) * P + p, ok ? double(jr[q].d[m]) : qnan);
      st_nt(jac + ((q + 3) * 7 + D::m0 + m) * P + p, ok ? double(jv[q].d[m]) : qnan);
    }
}

// One workgroup's satellite i: its points p0 + j for j < cnt at times tt[j],
// columns of P entries (dense: p0 = i T, tt = t; CSR: p0 = offsets[i], tt =
// t + p0).
template <class TS, class TP>
__device__ __forceinline__ void jac_sat(const RecordView& rv, int64_t n, const double* __restrict__ elem, int64_t i,
                                        int64_t p0, int64_t cnt, int64_t P, const double* __restrict__ tt,
                                        double* __restrict__ jac) {
  __shared__ double dc[7][kNRec];
  const uint32_t scode = rv.slots[i].info & kInfoCodeMask;
  if (threadIdx.x < 7) {
    const int m = threadIdx.x;
    if (scode == 0) {
      Dual1 el[7];
      for (int k = 0; k < 7; ++k) el[k] = Dual1(elem[k * n + i], k == m ? 1.0 : 0.0);
      GravIn gi{rv.hdr[kHRadius], rv.hdr[kHJ2], rv.hdr[kHJ4], rv.hdr[kHKe], rv.hdr[kHJ3oJ2]};
      Dual1 rec[kNRec];
      uint32_t code;
      bool isimp, dsp;
      init_record<Dual1>(gi, el, rec, &code, &isimp, &dsp);
#pragma unroll
      for (int k = 0; k < kNRec; ++k) dc[m][k] = k == kEpochMin ? 0.0 : rec[k].d;
    } else {
#pragma unroll
      for (int k = 0; k < kNRec; ++k) dc[m][k] = 0.0;
    }
  }
  __syncthreads();
  // the constants are read after the duals' registers are free again
  const SatC<TS, TP> c = load_sat<TS, TP, false>(rv, i);
  const Grav g = load_grav(rv);
  const double* t = tt;
  for (int64_t j = threadIdx.x; j < cnt; j += kVjpBlock) {
    const int64_t p = p0 + j;
    // the sensitivities are read from LDS where each step uses them: without
    // this fence the compiler would hoist all 238 loop-invariant loads into
    // registers ahead of the loop
    asm volatile("" ::: "memory");
    jacobian_pass<TS, TP, Dirs<0, 4>>(c, g, t[j], dc, jac, P, p);
    asm volatile("" ::: "memory");
    jacobian_pass<TS, TP, Dirs<4, 3>>(c, g, t[j], dc, jac, P, p);
  }
}

template <class TS, class TP>
__global__ void __launch_bounds__(kVjpBlock, kVjpBlocksPerCU<TP>)
    jacobian_kernel(RecordView rv, int64_t n, const double* __restrict__ elem, const double* __restrict__ t,
                    int64_t T, double* __restrict__ jac) {
  const int64_t i = blockIdx.x;
  jac_sat<TS, TP>(rv, n, elem, i, i * T, T, n * T, t, jac);
}

// CSR time lists, offsets clamped per workgroup as for the ragged VJP.
template <class TS, class TP>
__global__ void __launch_bounds__(kVjpBlock, kVjpBlocksPerCU<TP>)
    jacobian_ragged_kernel(RecordView rv, int64_t n, const double* __restrict__ elem,
                           const int64_t* __restrict__ offsets, const double* __restrict__ t, int64_t nnz,
                           double* __restrict__ jac) {
  const int64_t i = blockIdx.x;
  int64_t lo = offsets[i], hi = offsets[i + 1];
  lo = lo < 0 ? 0 : (lo > nnz ? nnz : lo);
  hi = hi < lo ? lo : (hi > nnz ? nnz : hi);
  jac_sat<TS, TP>(rv, n, elem, i, lo, hi - lo, nnz, t + lo, jac);
}

hipError_t launch_jacobian(int precision, int64_t n, const double* elem, const void* consts, const double* t,
                           int64_t T, double* jac, hipStream_t s) {
  const RecordView rv = view_of(consts, n);
  if (precision == 0)
    hipLaunchKernelGGL((jacobian_kernel<double, double>), dim3(unsigned(n)), dim3(kVjpBlock), 0, s, rv, n, elem, t, T,
                       jac);
  else if (precision == 2)
    hipLaunchKernelGGL((jacobian_kernel<double, float>), dim3(unsigned(n)), dim3(kVjpBlock), 0, s, rv, n, elem, t, T,
                       jac);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_vjp(int precision, int64_t n, const double* elem, const void* consts, const double* t, int64_t T,
                      const void* gr, const void* gv, double* gelem, hipStream_t s) {
  const RecordView rv = view_of(consts, n);
  if (precision == 0) {
    hipLaunchKernelGGL((vjp_kernel<double, double>), dim3(unsigned(n)), dim3(kVjpBlock), 0, s, rv, n, elem, t, T,
                       static_cast<const double*>(gr), static_cast<const double*>(gv), gelem);
  } else if (precision == 2) {
    hipLaunchKernelGGL((vjp_kernel<double, float>), dim3(unsigned(n)), dim3(kVjpBlock), 0, s, rv, n, elem, t, T,
                       static_cast<const float*>(gr), static_cast<const float*>(gv), gelem);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_jacobian_ragged(int precision, int64_t n, const double* elem, const void* consts,
                                  const int64_t* offsets, const double* t, int64_t nnz, double* jac, hipStream_t s) {
  const RecordView rv = view_of(consts, n);
  if (precision == 0) {
    hipLaunchKernelGGL((jacobian_ragged_kernel<double, double>), dim3(unsigned(n)), dim3(kVjpBlock), 0, s, rv, n,
                       elem, offsets, t, nnz, jac);
  } else if (precision == 2) {
    hipLaunchKernelGGL((jacobian_ragged_kernel<double, float>), dim3(unsigned(n)), dim3(kVjpBlock), 0, s, rv, n,
                       elem, offsets, t, nnz, jac);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vjp_ragged(int precision, int64_t n, const double* elem, const void* consts, const int64_t* offsets,
                             const double* t, int64_t nnz, const void* gr, const void* gv, double* gelem,
                             hipStream_t s) {
  const RecordView rv = view_of(consts, n);
  if (precision == 0) {
    hipLaunchKernelGGL((vjp_ragged_kernel<double, double>), dim3(unsigned(n)), dim3(kVjpBlock), 0, s, rv, n, elem,
                       offsets, t, nnz, static_cast<const double*>(gr), static_cast<const double*>(gv), gelem);
  } else if (precision == 2) {
    hipLaunchKernelGGL((vjp_ragged_kernel<double, float>), dim3(unsigned(n)), dim3(kVjpBlock), 0, s, rv, n, elem,
                       offsets, t, nnz, static_cast<const float*>(gr), static_cast<const float*>(gv), gelem);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sgp4mi

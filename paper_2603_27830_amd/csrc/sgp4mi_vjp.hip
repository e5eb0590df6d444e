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

template <class TS, class TP>
__global__ void __launch_bounds__(kVjpBlock, kVjpBlocksPerCU<TP>)
    vjp_kernel(RecordView rv, int64_t n, const double* __restrict__ elem, const double* __restrict__ t, int64_t T,
               const TP* __restrict__ gr, const TP* __restrict__ gv, double* __restrict__ gelem) {
  constexpr int kWaves = kVjpBlock / 64;
  __shared__ double part[kWaves][kNRec];
  __shared__ double cbar[kNRec];
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const SatC<TS, TP> c = load_sat<TS, TP, false>(rv, i);
  const Grav g = load_grav(rv);
  double acc[kNRec];
#pragma unroll
  for (int k = 0; k < kNRec; ++k) acc[k] = 0.0;
  const int64_t P = n * T;
  for (int64_t j = threadIdx.x; j < T; j += kVjpBlock) {
    const int64_t p = i * T + j;
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
    double out = 0.0;
    if ((c.info & kInfoCodeMask) == 0) {
      Dual1 el[7];
      for (int k = 0; k < 7; ++k) el[k] = Dual1(elem[k * n + i], k == m ? 1.0 : 0.0);
      const double R = rv.hdr[kHRadius];
      GravIn gi{R, rv.hdr[kHJ2], rv.hdr[kHJ4], rv.hdr[kHKe], rv.hdr[kHJ3oJ2]};
      Dual1 rec[kNRec];
      uint32_t code;
      bool isimp;
      init_record<Dual1>(gi, el, rec, &code, &isimp);
      for (int k = 0; k < kNRec; ++k)
        if (k != kEpochMin && cbar[k] != 0.0) out += cbar[k] * rec[k].d;
    }
    gelem[m * n + i] = out;
  }
}

// Jacobian of the dense propagation (paper section 5: the state's sensitivity
// to the elements, the state-transition and covariance use):
// jac[(c * 7 + m) * P + p] = d state_c / d theta_m at point p, c over r_x, r_y,
// r_z, v_x, v_y, v_z and m over the seven differentiated elements; NaN where
// the point's code is 1, 2, 4 or 7.  One workgroup per satellite: seven lanes
// first push the unit tangents of the elements through the initialisation
// (forward-mode duals) into the constants' sensitivities dc_k / dtheta_m (LDS);
// then, per point, each lane runs the reverse sweep once per state component
// (unit cotangent) and contracts the constants' adjoints with them.
template <class TS, class TP>
__global__ void __launch_bounds__(kVjpBlock, kVjpBlocksPerCU<TP>)
    jacobian_kernel(RecordView rv, int64_t n, const double* __restrict__ elem, const double* __restrict__ t,
                    int64_t T, double* __restrict__ jac) {
  __shared__ double dc[7][kNRec];
  const int64_t i = blockIdx.x;
  const uint32_t scode = rv.slots[i].info & kInfoCodeMask;
  if (threadIdx.x < 7) {
    const int m = threadIdx.x;
    if (scode == 0) {
      Dual1 el[7];
      for (int k = 0; k < 7; ++k) el[k] = Dual1(elem[k * n + i], k == m ? 1.0 : 0.0);
      GravIn gi{rv.hdr[kHRadius], rv.hdr[kHJ2], rv.hdr[kHJ4], rv.hdr[kHKe], rv.hdr[kHJ3oJ2]};
      Dual1 rec[kNRec];
      uint32_t code;
      bool isimp;
      init_record<Dual1>(gi, el, rec, &code, &isimp);
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
  const int64_t P = n * T;
  const double qnan = __builtin_nan("");
  for (int64_t j = threadIdx.x; j < T; j += kVjpBlock) {
    const int64_t p = i * T + j;
    const double tj = t[j];
#pragma unroll 1
    for (int comp = 0; comp < 6; ++comp) {
      TP gr[3], gv[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        gr[q] = comp == q ? TP(1) : TP(0);
        gv[q] = comp == q + 3 ? TP(1) : TP(0);
      }
      double cb[kNRec];
#pragma unroll
      for (int k = 0; k < kNRec; ++k) cb[k] = 0.0;
      const uint32_t code = point_vjp<TS, TP>(c, g, tj, gr, gv, cb);
      const bool ok = code == 0 || code == 6;
      // One element at a time, the sensitivities re-read from LDS (the empty
      // asm keeps the compiler from hoisting all 238 of them into registers).
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        asm volatile("" ::: "memory");
        double row = 0.0;
#pragma unroll
        for (int k = 0; k < kNRec; ++k) row = fma(cb[k], dc[m][k], row);
        st_nt(jac + (comp * 7 + m) * P + p, ok ? row : qnan);
      }
    }
  }
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

}  // namespace sgp4mi

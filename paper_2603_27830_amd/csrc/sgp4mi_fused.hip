// Elements to states in one launch: initialisation fused into propagation.
//
// jaxsgp4 traces initialisation and propagation into one function and maps it
// over satellites and times (paper sections 2.2 and 3.1); the two-stage path
// of this library instead writes a 512-byte record per satellite and reads it
// back.  For short time lists (a catalogue propagated to one or a few epochs)
// the record round trip and the second launch dominate, so this kernel keeps
// the record on chip:
//   workgroup = 64 satellites x tt times (tt <= kFusedTT), 64 * tt lanes;
//   wavefront 0 initialises the 64 satellites, one per lane, and leaves the
//   constants in LDS (tt = 1: in the lane's own registers);
//   every lane then propagates one (satellite, time) point, lanes ordered
//   satellite-major so the stores of a workgroup are contiguous when tt = T.
// Longer time lists take a grid of ceil(T / tt) workgroups per 64 satellites,
// each repeating the 64 initialisations (one wavefront of initialisation per
// tt wavefronts of propagation); the entry point sends such batches to the
// two-stage path when the caller supplies a record workspace.
#include "sgp4mi_initcore.h"
#include "sgp4mi_out.h"

namespace sgp4mi {

constexpr int kFusedTT = 16;

struct FusedArgs {
  int64_t n, T;
  const double* elem;   // [8][n]
  const double* t;      // [T]
  uint8_t* user_flags;  // nullable
  double mu, radius, j2, j3, j4;
  double ref_day;       // reference instant of the epoch row, days after JD 2415020.0
  uint32_t tt;
};

// The satellite's constants as the two-stage path reads them from its slot:
// the double values, and their float roundings for the float types.
template <class TS, class TP>
__device__ __forceinline__ SatC<TS, TP> sat_of(const double* x, uint32_t info, const double* deep) {
  SatC<TS, TP> c;
  c.M0 = TS(x[kM0]); c.Mdot = TS(x[kMdot]); c.argp0 = TS(x[kArgp0]); c.argpdot = TS(x[kArgpdot]);
  c.node0 = TS(x[kNode0]); c.nodedot = TS(x[kNodedot]); c.nodecf = TS(x[kNodecf]); c.C1 = TS(x[kC1]);
  c.bC4 = TS(x[kBC4]); c.t2cof = TS(x[kT2cof]); c.argpcof = TS(x[kArgpcof]); c.Mcof = TS(x[kMcof]);
  c.D2 = TS(x[kD2]); c.D3 = TS(x[kD3]); c.D4 = TS(x[kD4]); c.bC5 = TS(x[kBC5]); c.t3cof = TS(x[kT3cof]);
  c.t4cof = TS(x[kT4cof]); c.t5cof = TS(x[kT5cof]); c.n0pp = TS(x[kN0pp]); c.a0pp = TS(x[kA0pp]);
  c.e0 = TS(x[kE0]);
  c.epoch_min = x[kEpochMin];
  c.eta = TP(x[kEta]); c.dM0 = TP(x[kDM0]); c.sinM0 = TP(x[kSinM0]); c.aycof = TP(x[kAycof]);
  c.Lcof = TP(x[kLcof]); c.c41 = TP(x[kC41]); c.x1 = TP(x[kX1]); c.x7 = TP(x[kX7]); c.cosi = TP(x[kCosi]);
  c.sini = TP(x[kSini]); c.i0 = TP(x[kI0]);
  c.spA1 = TP(x[kSpA1]); c.spX1h = TP(x[kSpX1h]); c.spX1k = TP(x[kSpX1k]); c.spX7q = TP(x[kSpX7q]);
  c.spCN = TP(x[kSpCN]); c.spCI = TP(x[kSpCI]);
  c.pC1 = TP(x[kC1]); c.pbC4 = TP(x[kBC4]); c.pD2 = TP(x[kD2]); c.pD3 = TP(x[kD3]); c.pD4 = TP(x[kD4]);
  c.pbC5 = TP(x[kBC5]); c.pMcof = TP(x[kMcof]); c.pArgpcof = TP(x[kArgpcof]); c.pA0pp = TP(x[kA0pp]);
  c.pE0 = TP(x[kE0]);
  c.info = info;
  c.deep = deep;
  return c;
}

// Gravity scalars as the initialisation kernel writes them to the record
// header (the same expressions, so both paths see the same values).
__device__ __forceinline__ Grav grav_of(const FusedArgs& a) {
  Grav g;
  g.ke = 60.0 / sqrt(a.radius * a.radius * a.radius / a.mu);
  g.radius = a.radius;
  g.vkms = a.radius * g.ke / 60.0;
  g.k2 = 0.5 * a.j2;
  g.j3oj2 = (a.j3 == 0.0) ? 0.0 : a.j3 / a.j2;
  g.radius_f = float(a.radius);
  g.vkms_f = float(a.radius * g.ke / 60.0);
  g.k2_f = float(0.5 * a.j2);
  return g;
}

// Initialisation of satellite i into rec (kNRec doubles) and, for a
// propagated deep-space satellite, deep (kNDeep doubles); returns the info word.
__device__ __forceinline__ uint32_t init_sat(const FusedArgs& a, const Grav& g, int64_t i, double* rec, double* deep,
                                             bool write_flags) {
  double el[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) el[k] = a.elem[k * a.n + i];
  const double epoch = a.elem[7 * a.n + i];
  const double j3oj2 = (a.j3 == 0.0) ? 0.0 : a.j3 / a.j2;
  GravIn gi{a.radius, a.j2, a.j4, g.ke, j3oj2};
  uint32_t code;
  bool isimp, dsp;
  init_record<double>(gi, el, rec, &code, &isimp, &dsp);
  rec[kEpochMin] = 1440.0 * epoch;
  if (dsp && code == 0) init_deep(el, rec, g.ke, a.ref_day + epoch, deep);
  if (write_flags && a.user_flags) {
    uint8_t f = 0;
    if (dsp) f |= 1;
    if (isimp) f |= 2;
    if (code == 1 || code == 2) f |= 4;
    if (dsp && code == 0 && deep[kDRes] != 0.0) f |= 8;
    a.user_flags[i] = f;
  }
  return code | (isimp ? kInfoIsimp : 0u) | (dsp ? kInfoDeep : 0u);
}

// tt = 1: one wavefront per 64 satellites, each lane initialises and
// propagates its own satellite to the single time.
template <class TS, class TP, bool kOff32>
__global__ void __launch_bounds__(64) fused_one_kernel(FusedArgs a, Out<TP, kOff32> out) {
  const int64_t i = int64_t(blockIdx.x) * 64 + threadIdx.x;
  if (i >= a.n) return;
  const Grav g = grav_of(a);
  double rec[kNRec], deep[kNDeep];
  const uint32_t info = init_sat(a, g, i, rec, deep, true);
  const SatC<TS, TP> c = sat_of<TS, TP>(rec, info, deep);
  PointState<TP> s;
  const uint32_t code = (c.info & kInfoDeep) ? deep_point<TS, TP>(c, g, a.t[0], s) : sgp4_point<TS, TP>(c, g, a.t[0], s);
  out.put(i, code, s);
}

template <class TS, class TP, bool kOff32>
__global__ void __launch_bounds__(64 * kFusedTT) fused_kernel(FusedArgs a, Out<TP, kOff32> out) {
  __shared__ double lrec[kNRec][64];
  __shared__ double ldeep[64][kNDeep];
  __shared__ uint32_t linfo[64];
  const int64_t i0 = int64_t(blockIdx.x) * 64;
  const Grav g = grav_of(a);
  if (threadIdx.x < 64) {
    const int64_t i = i0 + threadIdx.x;
    if (i < a.n) {
      double rec[kNRec];
      const uint32_t info = init_sat(a, g, i, rec, ldeep[threadIdx.x], blockIdx.y == 0);
#pragma unroll
      for (int k = 0; k < kNRec; ++k) lrec[k][threadIdx.x] = rec[k];
      linfo[threadIdx.x] = info;
    }
  }
  __syncthreads();
  const uint32_t q = threadIdx.x;
  const uint32_t sl = q / a.tt;
  const int64_t i = i0 + sl;
  const int64_t j = int64_t(blockIdx.y) * a.tt + (q - sl * a.tt);
  if (i >= a.n || j >= a.T) return;
  double x[kNRec];
#pragma unroll
  for (int k = 0; k < kNRec; ++k) x[k] = lrec[k][sl];
  const SatC<TS, TP> c = sat_of<TS, TP>(x, linfo[sl], ldeep[sl]);
  PointState<TP> s;
  const uint32_t code = (c.info & kInfoDeep) ? deep_point<TS, TP>(c, g, a.t[j], s) : sgp4_point<TS, TP>(c, g, a.t[j], s);
  // kOff32: every point index is below 2^30 and fits 32-bit arithmetic
  out.put(kOff32 ? int64_t(uint32_t(i) * uint32_t(a.T) + uint32_t(j)) : i * a.T + j, code, s);
}

template <class TP>
static bool fused_fits32(int64_t P) {
  return P >= 0 && uint64_t(P) * sizeof(TP) < (uint64_t(1) << 32);
}

template <class TS, class TP, bool kOff32>
static void fused_go(const FusedArgs& a, void* r, void* v, uint8_t* err, hipStream_t s) {
  const int64_t P = a.n * a.T;
  Out<TP, kOff32> o{static_cast<TP*>(r), static_cast<TP*>(v), err, P};
  const unsigned gx = unsigned((a.n + 63) / 64);
  if (a.T == 1) {
    hipLaunchKernelGGL((fused_one_kernel<TS, TP, kOff32>), dim3(gx), dim3(64), 0, s, a, o);
    return;
  }
  const unsigned gy = unsigned((a.T + a.tt - 1) / a.tt);
  hipLaunchKernelGGL((fused_kernel<TS, TP, kOff32>), dim3(gx, gy), dim3(64 * a.tt), 0, s, a, o);
}

template <class TS, class TP>
static void fused_t(const FusedArgs& a, void* r, void* v, uint8_t* err, hipStream_t s) {
  if (fused_fits32<TP>(a.n * a.T)) fused_go<TS, TP, true>(a, r, v, err, s);
  else fused_go<TS, TP, false>(a, r, v, err, s);
}

// Largest T the fused grid covers (ceil(T / tt) workgroups in y).
int64_t fused_max_T() { return int64_t(65535) * kFusedTT; }

// Whether the fused grid's x extent (ceil(n / 64) workgroups of 64 tt lanes)
// fits a dispatch's 2^32 work-items.
bool fused_fits(int64_t n, int64_t T) {
  const uint64_t tt = uint64_t(T < kFusedTT ? T : kFusedTT);
  return grid_fits(uint64_t((n + 63) / 64), 64 * (tt > 0 ? tt : 1));
}

hipError_t launch_fused(int precision, const double g[5], double ref_day, int64_t n, const double* elem,
                        const double* t, int64_t T, void* r, void* v, uint8_t* err, uint8_t* user_flags,
                        hipStream_t s) {
  FusedArgs a;
  a.n = n;
  a.T = T;
  a.elem = elem;
  a.t = t;
  a.user_flags = user_flags;
  a.mu = g[0]; a.radius = g[1]; a.j2 = g[2]; a.j3 = g[3]; a.j4 = g[4];
  a.ref_day = ref_day;
  a.tt = uint32_t(T < kFusedTT ? T : kFusedTT);
  switch (precision) {
    case 0: fused_t<double, double>(a, r, v, err, s); break;
    case 1: fused_t<float, float>(a, r, v, err, s); break;
    case 2: fused_t<double, float>(a, r, v, err, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sgp4mi

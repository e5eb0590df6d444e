// Internal layout of the per-satellite constant record and device math helpers
// shared by the HIP translation units of the library.  Not a public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgp4mi {

// ------------------------------------------------------------------ record --
// The record produced by initialisation (the model's per-satellite constants,
// computed once and reused for every time; paper section 3.1 notes that the
// C++ baseline keeps initialisation separate while jaxsgp4 fuses it).
// Layout in device memory:
//   [header: 64 doubles]
//   [n slots of kSlotBytes = 512 bytes, one per satellite]:
//       bytes   0..319  kNRec doubles (full-precision constants)
//       bytes 320..479  kNRec floats  (the same constants rounded to float)
//       bytes 480..483  uint32 info: bits 0-7 satellite code, bit 8 isimp,
//                       bit 9 deep space
//       (entries ordered so that the FP32-mixed path touches two lines)
//   [n deep-space slots of kDeepBytes = 512 bytes, one per satellite]: the
//       lunar-solar secular rates, the long-period coefficients of the Sun and
//       the Moon and their mean anomalies at epoch, the tesseral resonance
//       terms (written and read only for satellites with the deep-space bit)
// One contiguous slot per satellite: a wavefront working on one satellite
// fetches its constants with a few wide loads from one base address.
// Order: the FP32-mixed near-Earth path reads the double copies of the first
// 13 entries (bytes 0-103 of the slot: one 128-byte line) and the float copies
// of entries 16-39 with the info word (bytes 384-483: another line), so a
// wavefront of that path fetches two of the slot's four lines.
enum Rec : int {
  // secular terms the mixed path keeps in double
  kM0, kMdot, kArgp0, kArgpdot, kNode0, kNodedot, kNodecf, kT2cof, kT3cof, kT4cof, kT5cof, kN0pp, kEpochMin,
  // read by FP64 only
  kC41, kX1, kX7,
  // taken in float by the mixed path
  kEta, kDM0, kSinM0, kAycof, kLcof, kCosi, kSini, kI0,
  // the short-period coefficients with k2 = J2 / 2 folded in (per point they
  // are multiplied by powers of 1 / p_L only): 1.5 k2 (3 cos^2 i - 1),
  // k2 / 2 sin^2 i, k2 sin^2 i, -k2 / 4 (7 cos^2 i - 1), 1.5 k2 cos i and
  // 1.5 k2 cos i sin i
  kSpA1, kSpX1h, kSpX1k, kSpX7q, kSpCN, kSpCI,
  // drag coefficients (the float paths' polynomials), mean a and e at epoch
  kC1, kBC4, kD2, kD3, kD4, kBC5, kMcof, kArgpcof, kA0pp, kE0,
  kNRec
};
static_assert(kEpochMin == 12 && kEta == 16 && kNRec == 40, "slot line layout");

// Header slots (doubles).
// kHF32: float copies of radius, velocity unit and k2 (three floats in the
// eight bytes of slots kHF32 and kHF32 + 1), so the float paths read them
// without a conversion per point.
// kHRefDay: the reference instant of the epoch row, in days after JD 2415020.0
// (1900 January 0.5, the origin of the lunar and solar arguments).
// kHGen, kHDeepGen: whether the record holds a deep-space satellite, without
// atomics or a clearing pass: every initialisation takes a fresh generation
// number g, the thread that writes the header stores g in kHGen and every
// deep-space satellite's thread stores g in kHDeepGen.  The two are equal if
// and only if this initialisation met a deep-space satellite (kHDeepGen can
// hold an older generation, never the current one otherwise; a stale equal
// value, possible only for a buffer reused across processes, just selects
// the general code path).
enum Hdr : int {
  kHMagic, kHN, kHNpad, kHKe, kHRadius, kHVkms, kHK2, kHJ2, kHJ3oJ2, kHJ4, kHMu, kHF32, kHRefDay = kHF32 + 2,
  kHGen, kHDeepGen,
  kHCount = 64
};
constexpr double kMagic = 20260331.0;

constexpr uint32_t kInfoCodeMask = 0xffu;
constexpr uint32_t kInfoIsimp = 0x100u;
constexpr uint32_t kInfoDeep = 0x200u;

// Deep-space slot: lunar-solar secular rates (rad/min), the Sun's and the
// Moon's mean anomalies at epoch, and per body (Sun, then Moon) the
// coefficients of the long-period terms of e, i, M, argp + cos i node and
// sin i node: the twice-anomaly pairs (x2, x3) and the body-eccentricity
// terms (l4, gh4).  Then the tesseral resonance: its class (0 none, 1 the
// 24 h class, 2 the 12 h class), the resonant mean longitude at epoch, its
// rate apart from the integrated mean motion, the Greenwich sidereal angle
// at epoch, and per term (24 h: 3, 12 h: 10) the pair (c cos phase,
// c sin phase) of its coefficient c and phase.
enum DeepRec : int {
  kDeDt, kDiDt, kDMDt, kDNodeDt, kDArgpDt, kDMb0, kDMb1,
  kDPer0 = 7,  // per body k: kDPer0 + 12 k + one of the offsets below
  kDRes = kDPer0 + 24, kDXlamo, kDXfact, kDGsto,
  kDRc0,  // term m: kDRc0 + 2 m (cos part), kDRc0 + 2 m + 1 (sin part)
  kNDeep = kDRc0 + 20
};
enum DeepPer : int { kPe2, kPe3, kPi2, kPi3, kPl2, kPl3, kPl4, kPgh2, kPgh3, kPgh4, kPh2, kPh3, kNPer };
// The Earth's rotation rate (rad/min) of the resonance; the resonance
// integrator's step and its reach from epoch (10 Julian years), in minutes.
constexpr double kEarthRot = 4.37526908801129966e-3;
constexpr double kResStepMin = 720.0;
constexpr double kResMaxMin = 5259600.0;
constexpr int kDeepBytes = 512;
struct alignas(16) DeepSlot {
  double d[kDeepBytes / 8];
};
static_assert(kNDeep * 8 <= kDeepBytes, "deep-space slot overflow");

// Point code of a ragged point that the offsets place in no satellite's list
// (malformed offsets given to the plan-less ragged call); r and v are NaN.
constexpr uint32_t kCodeUnowned = 8u;

constexpr int kSlotBytes = 512;
constexpr int kSlotF32 = kNRec * 8;            // byte offset of the float copies
constexpr int kSlotInfo = kSlotF32 + kNRec * 4;  // byte offset of the info word
static_assert(kSlotInfo + 4 <= kSlotBytes, "record slot overflow");

struct alignas(16) Slot {
  double d[kNRec];
  float f[kNRec];
  uint32_t info;
  uint32_t pad[(kSlotBytes - kSlotInfo - 4) / 4];
};
static_assert(sizeof(Slot) == kSlotBytes, "slot size");

// A dispatch's extent in work-items is a 32-bit number per grid dimension:
// groups * block must stay below 2^32 (not only groups below 2^31).
inline bool grid_fits(uint64_t groups, uint64_t block) { return groups * block <= 0xffffffffull; }

inline int64_t npad_of(int64_t n) { return (n + 63) / 64 * 64; }
inline size_t record_bytes(int64_t n) {
  return size_t(kHCount) * 8 + size_t(kSlotBytes + kDeepBytes) * size_t(n > 0 ? n : 0);
}

struct RecordView {
  const double* hdr;
  const Slot* slots;
  const DeepSlot* deep;
};

// Whether the record's initialisation met a deep-space satellite (see
// kHGen); read through the constant address space (scalar loads of two
// header words every wavefront shares).
__device__ __forceinline__ bool record_has_deep(const RecordView& rv) {
  typedef const __attribute__((address_space(4))) double* CHdrD;
  const CHdrD h = (CHdrD)rv.hdr;
  return h[kHGen] == h[kHDeepGen];
}

inline RecordView view_of(const void* base, int64_t n) {
  RecordView v;
  const char* b = static_cast<const char*>(base);
  v.hdr = reinterpret_cast<const double*>(b);
  v.slots = reinterpret_cast<const Slot*>(b + kHCount * 8);
  v.deep = reinterpret_cast<const DeepSlot*>(b + kHCount * 8 + size_t(kSlotBytes) * size_t(n > 0 ? n : 0));
  return v;
}

// Gravity-derived scalars read by the kernels (from the record header).
struct Grav {
  double ke, radius, vkms, k2, j3oj2;
  float radius_f, vkms_f, k2_f;
};
template <class T> __device__ __forceinline__ T grav_radius(const Grav& g);
template <class T> __device__ __forceinline__ T grav_vkms(const Grav& g);
template <class T> __device__ __forceinline__ T grav_k2(const Grav& g);
template <> __device__ __forceinline__ double grav_radius<double>(const Grav& g) { return g.radius; }
template <> __device__ __forceinline__ double grav_vkms<double>(const Grav& g) { return g.vkms; }
template <> __device__ __forceinline__ double grav_k2<double>(const Grav& g) { return g.k2; }
template <> __device__ __forceinline__ float grav_radius<float>(const Grav& g) { return g.radius_f; }
template <> __device__ __forceinline__ float grav_vkms<float>(const Grav& g) { return g.vkms_f; }
template <> __device__ __forceinline__ float grav_k2<float>(const Grav& g) { return g.k2_f; }

// ------------------------------------------------------------- math (FP64) --
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kInvTwoPi = 0.15915494309189533577;

// x - 2*pi*round(x / 2*pi): a representative of x mod 2*pi in about [-pi, pi].
__device__ __forceinline__ double wrap_pi(double x) { return fma(-kTwoPi, rint(x * kInvTwoPi), x); }

// Non-temporal stores: outputs are written once and never re-read by the kernel.
template <class T>
__device__ __forceinline__ void st_nt(T* p, T x) { __builtin_nontemporal_store(x, p); }

}  // namespace sgp4mi

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
// Layout in device memory, all SoA with a row stride of npad = round_up(n, 64):
//   [header: 64 doubles]
//   [f64 rows: kNRec x npad doubles]   full-precision constants
//   [f32 rows: kNRec x npad floats]    the same constants rounded to float
//   [info:     npad uint32]            bits 0-7 satellite code, bit 8 isimp
enum Rec : int {
  kM0, kMdot, kArgp0, kArgpdot, kNode0, kNodedot, kNodecf, kC1, kBC4, kT2cof,
  kArgpcof, kEta, kMcof, kDM0, kD2, kD3, kD4, kBC5, kSinM0, kT3cof, kT4cof, kT5cof,
  kN0pp, kA0pp, kE0, kAycof, kLcof, kC41, kX1, kX7, kCosi, kSini, kI0, kEpochMin,
  kNRec
};

// Header slots (doubles).
enum Hdr : int { kHMagic, kHN, kHNpad, kHKe, kHRadius, kHVkms, kHK2, kHJ2, kHJ3oJ2, kHJ4, kHMu, kHCount = 64 };
constexpr double kMagic = 20260331.0;

constexpr uint32_t kInfoCodeMask = 0xffu;
constexpr uint32_t kInfoIsimp = 0x100u;

inline int64_t npad_of(int64_t n) { return (n + 63) / 64 * 64; }
inline size_t record_bytes(int64_t n) {
  const int64_t np = npad_of(n);
  return size_t(kHCount) * 8 + size_t(kNRec) * 8 * np + size_t(kNRec) * 4 * np + 4 * np;
}

struct RecordView {
  const double* hdr;
  const double* f64;   // row k at f64 + k * npad
  const float* f32;    // row k at f32 + k * npad
  const uint32_t* info;
  int64_t npad;
};

inline RecordView view_of(const void* base, int64_t n) {
  RecordView v;
  const int64_t np = npad_of(n);
  const char* b = static_cast<const char*>(base);
  v.hdr = reinterpret_cast<const double*>(b);
  v.f64 = reinterpret_cast<const double*>(b + kHCount * 8);
  v.f32 = reinterpret_cast<const float*>(b + kHCount * 8 + size_t(kNRec) * 8 * np);
  v.info = reinterpret_cast<const uint32_t*>(b + kHCount * 8 + size_t(kNRec) * 12 * np);
  v.npad = np;
  return v;
}

// Gravity-derived scalars read by the kernels (from the record header).
struct Grav {
  double ke, radius, vkms, k2;
};

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

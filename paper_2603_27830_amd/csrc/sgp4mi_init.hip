// Initialisation kernel: mean elements -> per-satellite constant record.
//
// One lane per satellite, double precision; the model's steps are in
// sgp4mi_initcore.h (shared with the derivative kernel of the VJP).
#include <atomic>
#include <chrono>

#include "sgp4mi_initcore.h"

namespace sgp4mi {

struct InitArgs {
  int64_t n, npad;
  const double* elem;   // [8][n]
  double* hdr;
  Slot* slots;
  DeepSlot* deep;
  uint8_t* user_flags;  // nullable
  double mu, radius, j2, j3, j4;
  double ref_day;       // reference instant of the epoch row, days after JD 2415020.0
  double gen;           // this initialisation's generation number (kHGen)
};

// kStaged: the 64 records of the workgroup are assembled in LDS and copied
// out as one contiguous run of 64 slots (each store instruction of the
// wavefront writes 1 KiB of consecutive bytes), instead of each lane writing
// its own 512-byte slot (each store instruction touching 64 cache lines).
template <bool kStaged>
__global__ void __launch_bounds__(64) init_kernel(InitArgs a) {
  __shared__ Slot stage[kStaged ? 64 : 1];
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
    h[kHRefDay] = a.ref_day;
    h[kHGen] = a.gen;
    float* hf = reinterpret_cast<float*>(h + kHF32);
    hf[0] = float(a.radius);
    hf[1] = float(a.radius * ke / 60.0);
    hf[2] = float(0.5 * a.j2);
    hf[3] = 0.0f;
  }
  const int64_t n = a.n;
  const int64_t i0 = int64_t(blockIdx.x) * blockDim.x;
  if (!kStaged && i >= n) return;
  if (i < n) {
    double el[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) el[k] = a.elem[k * n + i];
    const double epoch = a.elem[7 * n + i];
    GravIn gi{a.radius, a.j2, a.j4, ke, j3oj2};
    double rec[kNRec];
    uint32_t code;
    bool isimp, deep;
    init_record<double>(gi, el, rec, &code, &isimp, &deep);
    bool resonant = false;
    if (deep && code == 0) {
      double d[kNDeep];
      init_deep(el, rec, ke, a.ref_day + epoch, d);
      resonant = d[kDRes] != 0.0;
#pragma unroll
      for (int k = 0; k < kNDeep; ++k) a.deep[i].d[k] = d[k];
    }
    rec[kEpochMin] = 1440.0 * epoch;
    Slot* slot = kStaged ? &stage[threadIdx.x] : a.slots + i;
#pragma unroll
    for (int k = 0; k < kNRec; ++k) {
      slot->d[k] = rec[k];
      slot->f[k] = float(rec[k]);
    }
    slot->info = code | (isimp ? kInfoIsimp : 0u) | (deep ? kInfoDeep : 0u);
    if (deep) a.hdr[kHDeepGen] = a.gen;  // every such thread stores the same value
    if (a.user_flags) {
      uint8_t f = 0;
      if (deep) f |= 1;
      if (resonant) f |= 8;
      if (isimp) f |= 2;
      if (code == 1 || code == 2) f |= 4;
      a.user_flags[i] = f;
    }
  }
  if (kStaged) {
    __syncthreads();
    // Copy the workgroup's valid slots (whole 16-byte chunks) to device memory.
    const int64_t valid = n - i0 < 64 ? n - i0 : 64;
    const int chunks = int(valid) * (kSlotBytes / 16);
    const uint4* src = reinterpret_cast<const uint4*>(stage);
    uint4* dst = reinterpret_cast<uint4*>(a.slots + i0);
    for (int c = threadIdx.x; c < chunks; c += 64) dst[c] = src[c];
  }
}

// Catalogues from this size on take the staged kernel (its copy-out adds
// latency that a few hundred workgroups do not hide).
constexpr int64_t kInitStagedFrom = 65536;

// Generation numbers of initialisations: process-wide and increasing, seeded
// from the clock so that a record buffer reused by another process rarely
// meets its old value (which would only select the general code path).
static double next_generation() {
  static std::atomic<uint64_t> counter{uint64_t(std::chrono::steady_clock::now().time_since_epoch().count()) &
                                       ((uint64_t(1) << 40) - 1)};
  return double(++counter);  // below 2^41: exact in a double
}

hipError_t launch_init(const double g[5], double ref_day, int64_t n, const double* elem, void* consts,
                       uint8_t* user_flags, hipStream_t s) {
  InitArgs a;
  a.n = n;
  a.npad = npad_of(n);
  a.elem = elem;
  char* b = static_cast<char*>(consts);
  a.hdr = reinterpret_cast<double*>(b);
  a.slots = reinterpret_cast<Slot*>(b + kHCount * 8);
  a.deep = reinterpret_cast<DeepSlot*>(b + kHCount * 8 + size_t(kSlotBytes) * size_t(n));
  a.ref_day = ref_day;
  a.gen = next_generation();
  a.user_flags = user_flags;
  a.mu = g[0]; a.radius = g[1]; a.j2 = g[2]; a.j3 = g[3]; a.j4 = g[4];
  const int64_t blocks = (n + 63) / 64;  // 64-wide: a short kernel spread over more compute units
  if (n >= kInitStagedFrom)
    hipLaunchKernelGGL(init_kernel<true>, dim3(unsigned(blocks)), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(init_kernel<false>, dim3(unsigned(blocks > 0 ? blocks : 1)), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace sgp4mi

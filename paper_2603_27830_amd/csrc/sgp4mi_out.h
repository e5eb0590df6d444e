// Output writer shared by the propagation kernels: component-major SoA
// arrays r[c * P + p], v[c * P + p] and the code array err[p]; codes 1, 2, 4
// and 7 write NaN states.
//
// Store policy (measured on MI355X): the state components go out as
// non-temporal stores (a wavefront writes 256 or 512 contiguous bytes per
// component); the one-byte codes as ordinary stores, which the L2 merges into
// whole lines before they reach HBM (a wavefront's 64 code bytes rarely fill
// an aligned line, and written past the cache each such piece is a partial
// write): 9,341 x 1,000 mixed 64 -> 60 us, FP32 67 -> 63 us, the 1M ragged
// catalogue mixed 5.09 -> 4.74 ms, FP64 unchanged.
#pragma once

#include "sgp4mi_point.h"

namespace sgp4mi {

// Output writer: six component arrays and the code array.  With kOff32 the
// per-lane offset is a 32-bit byte offset from uniform base pointers (valid
// when each component array is below 4 GiB), so each store takes its base
// from scalar registers and no 64-bit address arithmetic per store.
template <class TP, bool kOff32>
struct Out {
  TP* r;
  TP* v;
  uint8_t* err;
  int64_t P;
  __device__ __forceinline__ void put(int64_t p, uint32_t code, const PointState<TP>& s) const {
    // Codes 1, 2, 4 and 7 carry no state: such lanes (rare, and usually whole
    // satellites) overwrite the values with NaN in their own block, so the
    // common path copies nothing.
    TP x0 = s.r[0], x1 = s.r[1], x2 = s.r[2], y0 = s.v[0], y1 = s.v[1], y2 = s.v[2];
    if (!s.ok) {
      // The empty asm keeps the branch around this block: the block is then
      // skipped whenever no lane of the wavefront takes it.
      asm volatile("");
      const TP q = TP(__builtin_nan(""));
      x0 = q; x1 = q; x2 = q; y0 = q; y1 = q; y2 = q;
    }
    store(p, code, x0, x1, x2, y0, y1, y2);
  }
  __device__ __forceinline__ void store(int64_t p, uint32_t code, TP x0, TP x1, TP x2, TP y0, TP y1, TP y2) const {
    if (kOff32) {
      const uint32_t off = uint32_t(p) * uint32_t(sizeof(TP));
      char* rb = reinterpret_cast<char*>(r);
      char* vb = reinterpret_cast<char*>(v);
      const size_t stride = size_t(P) * sizeof(TP);
      st_nt(reinterpret_cast<TP*>(rb + off), x0);
      st_nt(reinterpret_cast<TP*>(rb + stride + off), x1);
      st_nt(reinterpret_cast<TP*>(rb + 2 * stride + off), x2);
      st_nt(reinterpret_cast<TP*>(vb + off), y0);
      st_nt(reinterpret_cast<TP*>(vb + stride + off), y1);
      st_nt(reinterpret_cast<TP*>(vb + 2 * stride + off), y2);
      // the code array seen in the global address space: the store then takes
      // its base from scalar registers and the 32-bit offset as it is
      typedef __attribute__((address_space(1))) uint8_t* GByte;
      *((GByte)err + uint32_t(p)) = uint8_t(code);
    } else {
      st_nt(r + p, x0);
      st_nt(r + P + p, x1);
      st_nt(r + 2 * P + p, x2);
      st_nt(v + p, y0);
      st_nt(v + P + p, y1);
      st_nt(v + 2 * P + p, y2);
      err[p] = uint8_t(code);
    }
  }
};

}  // namespace sgp4mi

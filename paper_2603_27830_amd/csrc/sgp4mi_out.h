// Output writer shared by the propagation kernels: component-major SoA
// arrays r[c * P + p], v[c * P + p] and the code array err[p], written with
// non-temporal stores; codes 1, 2, 4 and 7 write NaN states.
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
    // satellites) take their own store path instead of a select per component.
    if (code != 0 && code != 6) {
      const TP q = TP(__builtin_nan(""));
      store(p, code, q, q, q, q, q, q);
    } else {
      store(p, code, s.r[0], s.r[1], s.r[2], s.v[0], s.v[1], s.v[2]);
    }
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
      st_nt(err + uint32_t(p), uint8_t(code));
    } else {
      st_nt(r + p, x0);
      st_nt(r + P + p, x1);
      st_nt(r + 2 * P + p, x2);
      st_nt(v + p, y0);
      st_nt(v + P + p, y1);
      st_nt(v + 2 * P + p, y2);
      st_nt(err + p, uint8_t(code));
    }
  }
};

}  // namespace sgp4mi

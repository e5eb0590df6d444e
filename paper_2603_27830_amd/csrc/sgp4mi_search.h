// Owner search of the ragged flat mapping: which satellite's time list holds
// point p of a CSR batch (satellite i owns points offsets[i] .. offsets[i+1]).
//
// Host and device code: the kernels call it with a wavefront ballot, the CPU
// tests with a 64-lane loop and a bounds-checked offsets array.  Nothing here
// depends on the offsets being well formed: for ANY int64 offsets[0..n] with
// n >= 1, every index read lies in [0, n], the search ends after at most
// ceil(log64(n)) + 1 rounds, and the returned satellite lies in [0, n).  Only
// whether the point really belongs to that satellite depends on the offsets;
// point_owner reports it.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define SGP4MI_HD __host__ __device__
#else
#define SGP4MI_HD
#endif

namespace sgp4mi {

// Index of the highest set bit of a non-zero mask.
SGP4MI_HD inline int top_bit(uint64_t m) { return 63 - __builtin_clzll(m); }

// 64-way search for the largest i in [0, n) with offsets[i] <= q, by rounds in
// which lane l probes index lo + l * step of [lo, hi).  probe(lo, step, hi)
// returns the mask of lanes l with lo + l * step < hi and offsets[lo + l *
// step] <= q.  For non-decreasing offsets with offsets[0] <= q the passing
// lanes form a prefix and the result is exact.  Otherwise: an empty mask
// (possible only in the first round, when offsets[0] > q) ends the search at
// lo = 0; a mask with holes keeps its highest lane, whose index passed, so lo
// stays in [0, hi) and [lo, hi) shrinks to at most ceil((hi - lo) / 64).
template <class Probe>
SGP4MI_HD inline int64_t wave_search(int64_t n, const Probe& probe) {
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) >> 6;
    const uint64_t mask = probe(lo, step, hi);
    if (mask == 0) break;
    const int64_t nlo = lo + step * top_bit(mask);
    hi = nlo + step < hi ? nlo + step : hi;
    lo = nlo;
  }
  return lo;
}

// From first, the owner of an earlier point of the same or a preceding 64-point
// chunk (or any index in [0, n)), walk forward over the satellites whose lists
// end at or before p.  Returns the satellite in [0, n) where the walk stops and
// sets *owned when offsets[sat] <= p < offsets[sat + 1], i.e. the point lies
// in that satellite's list.  With well-formed offsets (offsets[0] = 0,
// non-decreasing, offsets[n] = nnz > p) and first from wave_search of a q <= p,
// the point is always owned.
template <class Off>
SGP4MI_HD inline int64_t point_owner(const Off& offsets, int64_t n, int64_t first, int64_t p, bool* owned) {
  int64_t sat = first < 0 ? 0 : (first >= n ? n - 1 : first);
  while (sat + 1 < n && offsets[sat + 1] <= p) ++sat;
  *owned = offsets[sat] <= p && p < offsets[sat + 1];
  return sat;
}

}  // namespace sgp4mi

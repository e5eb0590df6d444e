// CPU check of the ragged owner search (sgp4mi_search.h) over random and
// adversarial int64 offsets.  Built with g++ and the address and undefined-
// behaviour sanitizers; the offsets are read through a bounds-checked view, so
// any index outside [0, n] aborts.  Exit status 0 and a summary line on
// success.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "sgp4mi_search.h"

namespace {

struct Checked {
  const std::vector<int64_t>* v;
  int64_t operator[](int64_t i) const {
    if (i < 0 || i >= int64_t(v->size())) {
      std::fprintf(stderr, "out-of-range offsets read: index %lld of %zu\n", (long long)i, v->size());
      std::abort();
    }
    return (*v)[size_t(i)];
  }
};

int64_t g_rounds_max = 0;
int64_t g_checked = 0, g_owned = 0, g_unowned = 0;

int rounds_bound(int64_t n) {
  int r = 1;
  for (int64_t span = 1; span < n; span *= 64) ++r;
  return r;
}

// One batch: every chunk of 64 points of [0, nnz), every lane of it.
void run(const std::vector<int64_t>& off, int64_t nnz, bool well_formed, int64_t max_chunks = 1 << 14) {
  const int64_t n = int64_t(off.size()) - 1;
  const Checked c{&off};
  const int64_t nchunks = (nnz + 63) / 64;
  const int64_t stride = nchunks > max_chunks ? nchunks / max_chunks : 1;
  for (int64_t k = 0; k < nchunks; k += stride) {
    const int64_t q = k * 64;
    int rounds = 0;
    auto probe = [&](int64_t lo, int64_t step, int64_t hi) {
      ++rounds;
      if (!(0 <= lo && lo < hi && hi <= n && step >= 1)) {
        std::fprintf(stderr, "bad probe range lo=%lld hi=%lld step=%lld n=%lld\n", (long long)lo, (long long)hi,
                     (long long)step, (long long)n);
        std::abort();
      }
      uint64_t m = 0;
      for (int lane = 0; lane < 64; ++lane) {
        const int64_t idx = lo + step * lane;
        if (idx < hi && c[idx] <= q) m |= uint64_t(1) << lane;
      }
      return m;
    };
    const int64_t first = sgp4mi::wave_search(n, probe);
    if (first < 0 || first >= n) { std::fprintf(stderr, "search result %lld outside [0, %lld)\n", (long long)first, (long long)n); std::abort(); }
    if (rounds > rounds_bound(n)) { std::fprintf(stderr, "search took %d rounds for n=%lld\n", rounds, (long long)n); std::abort(); }
    g_rounds_max = std::max<int64_t>(g_rounds_max, rounds);
    for (int lane = 0; lane < 64; ++lane) {
      const int64_t p = q + lane;
      if (p >= nnz) break;
      bool owned = false;
      const int64_t sat = sgp4mi::point_owner(c, n, first, p, &owned);
      ++g_checked;
      if (sat < 0 || sat >= n) { std::fprintf(stderr, "owner %lld outside [0, %lld)\n", (long long)sat, (long long)n); std::abort(); }
      if (owned != (off[size_t(sat)] <= p && p < off[size_t(sat) + 1])) { std::fprintf(stderr, "owned flag wrong\n"); std::abort(); }
      owned ? ++g_owned : ++g_unowned;
      if (well_formed) {
        // the unique satellite with off[i] <= p < off[i+1]: last i with off[i] <= p
        const int64_t want = int64_t(std::upper_bound(off.begin(), off.end(), p) - off.begin()) - 1;
        if (!owned || sat != want) {
          std::fprintf(stderr, "well-formed offsets: point %lld got %lld (owned %d), want %lld\n", (long long)p,
                       (long long)sat, int(owned), (long long)want);
          std::abort();
        }
      }
    }
  }
}

std::vector<int64_t> csr(const std::vector<int64_t>& lens) {
  std::vector<int64_t> off(lens.size() + 1, 0);
  for (size_t i = 0; i < lens.size(); ++i) off[i + 1] = off[i] + lens[i];
  return off;
}

}  // namespace

int main() {
  std::mt19937_64 rng(20260331);
  const int64_t kMin = std::numeric_limits<int64_t>::min(), kMax = std::numeric_limits<int64_t>::max();
  int cases = 0;

  // Well-formed: random lengths including empty lists, one satellite, long runs of empties.
  for (int64_t n : {1, 2, 3, 63, 64, 65, 100, 4095, 4096, 4097, 300000}) {
    for (int kind = 0; kind < 4; ++kind) {
      std::vector<int64_t> lens(static_cast<size_t>(n));
      for (auto& L : lens) {
        const uint64_t u = rng();
        L = kind == 0 ? int64_t(u % 300) : kind == 1 ? (u % 4 ? 0 : int64_t(u % 200)) : kind == 2 ? 1 : int64_t(u % 5000 == 0 ? 10000 : 0);
      }
      if (kind == 3) lens[size_t(n - 1)] += 70;
      const auto off = csr(lens);
      if (off.back() == 0) continue;
      run(off, off.back(), true);
      ++cases;
    }
  }

  // Malformed: offsets[0] > 0; offsets[n] != nnz; decreasing steps; random junk; int64 extremes.
  for (int64_t n : {1, 2, 5, 64, 65, 1000, 70000}) {
    for (int kind = 0; kind < 9; ++kind) {
      std::vector<int64_t> off(static_cast<size_t>(n) + 1);
      int64_t nnz = 0;
      if (kind == 0) {  // shifted start
        std::vector<int64_t> lens(size_t(n), 7);
        off = csr(lens);
        nnz = off.back();
        for (auto& o : off) o += 100;
      } else if (kind == 1) {  // ends short of nnz
        std::vector<int64_t> lens(size_t(n), 9);
        off = csr(lens);
        nnz = off.back() + 500;
      } else if (kind == 2) {  // ends beyond nnz
        std::vector<int64_t> lens(size_t(n), 9);
        off = csr(lens);
        nnz = off.back() / 2 + 1;
      } else if (kind == 3) {  // one decreasing step in the middle
        std::vector<int64_t> lens(size_t(n), 11);
        off = csr(lens);
        nnz = off.back();
        off[size_t(n / 2)] = nnz + 1000;
      } else if (kind == 4) {  // uniform random junk
        for (auto& o : off) o = int64_t(rng() % 100000) - 1000;
        nnz = 50000;
      } else if (kind == 5) {  // full-range junk
        for (auto& o : off) o = int64_t(rng());
        nnz = 40000;
      } else if (kind == 6) {  // extremes
        for (size_t i = 0; i < off.size(); ++i) off[i] = (i % 3 == 0) ? kMin : (i % 3 == 1 ? kMax : 0);
        nnz = 10000;
      } else if (kind == 7) {  // everything at kMax
        for (auto& o : off) o = kMax;
        nnz = 3000;
      } else {  // everything at kMin (non-decreasing, but offsets[n] != nnz)
        for (auto& o : off) o = kMin;
        nnz = 3000;
      }
      run(off, nnz, false);
      ++cases;
    }
  }
  std::printf("ok: %d offset arrays, %lld points checked (%lld owned, %lld unowned), at most %lld search rounds\n",
              cases, (long long)g_checked, (long long)g_owned, (long long)g_unowned, (long long)g_rounds_max);
  return 0;
}

// Propagation kernels: dense N x T grids and ragged CSR time lists.
//
// One lane per (satellite, time) point (paper section 2.2: the two independent
// axes of parallelism, satellites and times).  Three mappings:
//   dense      block = (satellite, run of times); the satellite is uniform
//              over the block, so its constants are scalar loads.
//   tiles      ragged lists cut into tiles of <= 64 points of one satellite,
//              one tile per wavefront, persistent grid-stride loop.
//   flat       ragged lists read as one flat run of points, 64 per wavefront;
//              each lane finds its satellite from the tile's first satellite
//              by a short forward scan of the offsets (constants per lane).
// Outputs are component-major SoA, r[c * P + p] (states by non-temporal
// stores, codes by ordinary ones); codes 1, 2, 4 and 7 write NaN states.
#include "sgp4mi_out.h"
#include "sgp4mi_search.h"

namespace sgp4mi {

// Register budget of the one-wavefront-per-tile kernels (the default dense and
// ragged launches): the deep-space branch, taken by whole wavefronts of
// deep-space satellites, holds more values than the near-Earth path and would
// otherwise set every wavefront's allocation (74 registers, six wavefronts per
// SIMD); asking for at least seven keeps eight, with the near-Earth path
// compiled to the instructions it has without the branch.
#define SGP4MI_TILE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(7, 8)))

// ------------------------------------------------------------------ dense --
// Grid (n, ceil(T / kBlock)): one point per lane.  When T needs more than
// 65535 workgroups in y, kLoop makes each lane stride over the remaining times.
template <class TS, class TP, int kBlock, bool kVec, bool kOff32, bool kLoop>
__global__ void __launch_bounds__(kBlock) dense_kernel(RecordView rv, const double* __restrict__ t, int64_t T,
                                                       Out<TP, kOff32> out) {
  const int64_t i = blockIdx.x;
  int64_t j = int64_t(blockIdx.y) * kBlock + threadIdx.x;
  if (!kLoop) {
    if (j >= T) return;
    const Grav g = load_grav(rv);
    PointState<TP> s;
    const uint32_t code = propagate_point<TS, TP, kVec>(rv, i, g, t[j], s);
    out.put(i * T + j, code, s);
    return;
  }
  const Grav g = load_grav(rv);
  for (; j < T; j += int64_t(gridDim.y) * kBlock) {
    PointState<TP> s;
    const uint32_t code = propagate_point<TS, TP, kVec>(rv, i, g, t[j], s);
    out.put(i * T + j, code, s);
  }
}

// Tile variant: one wavefront per tile of 64 times of one satellite (tile w =
// satellite w / tps, times 64 * (w % tps) ...), workgroups of kBlock / 64
// independent wavefronts, no loop.  Tile indices fit 32 bits (checked by the
// launcher).
template <class TS, class TP, int kBlock, bool kOff32>
__global__ void __launch_bounds__(kBlock) SGP4MI_TILE_OCCUPANCY dense_tile_kernel(RecordView rv, const double* __restrict__ t, int64_t T,
                                                            uint32_t tps, uint32_t ntiles, Out<TP, kOff32> out) {
  constexpr int kWaves = kBlock / 64;
  const uint32_t w = blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= ntiles) return;
  const uint32_t sat = w / tps;
  const int64_t j = int64_t(w - sat * tps) * 64 + (threadIdx.x & 63);
  if (j >= T) return;
  const Grav g = load_grav(rv);
  PointState<TP> s;
  const uint32_t code = propagate_point<TS, TP, false>(rv, int64_t(sat), g, t[j], s);
  // kOff32: every point index is below 2^30, so the index is formed in 32 bits
  // (the satellite's row start on the scalar unit, one vector add)
  const int64_t p = kOff32 ? int64_t(uint32_t(sat) * uint32_t(T) + uint32_t(j)) : int64_t(sat) * T + j;
  out.put(p, code, s);
}

// Flat variant for short time lists: lane p -> satellite p / T, time p % T,
// so every lane of a wavefront has a point however short the list; each lane
// reads its satellite's constants with vector loads.
template <class TS, class TP, int kBlock, bool kOff32>
__global__ void __launch_bounds__(kBlock) dense_flat_kernel(RecordView rv, const double* __restrict__ t, int64_t T,
                                                            Out<TP, kOff32> out) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= out.P) return;
  int64_t i, j;
  if (kOff32) {  // P < 2^32: 32-bit division
    const uint32_t i32 = uint32_t(p) / uint32_t(T);
    i = i32;
    j = int64_t(uint32_t(p) - i32 * uint32_t(T));
  } else {
    i = p / T;
    j = p - i * T;
  }
  const Grav g = load_grav(rv);
  PointState<TP> s;
  const uint32_t code = propagate_point<TS, TP, true>(rv, i, g, t[j], s);
  out.put(p, code, s);
}

// Persistent variant: a fixed grid; each wavefront walks tiles of 64 times of
// one satellite (tile w = satellite w / tps, times 64 * (w % tps) ...), so no
// workgroup is dispatched per satellite and a wavefront's consecutive tiles
// usually share the satellite's constants in cache.
template <class TS, class TP, int kBlock, bool kVec, bool kOff32>
__global__ void __launch_bounds__(kBlock) dense_persistent_kernel(RecordView rv, const double* __restrict__ t,
                                                                  int64_t T, uint32_t tps, uint64_t ntiles,
                                                                  Out<TP, kOff32> out) {
  constexpr int kWaves = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const uint64_t wave0 = uint64_t(blockIdx.x) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t nwaves = uint64_t(gridDim.x) * kWaves;
  const Grav g = load_grav(rv);
  for (uint64_t w = wave0; w < ntiles; w += nwaves) {
    const uint64_t sat = w / tps;
    const int64_t j = int64_t(w - sat * tps) * 64 + lane;
    if (j < T) {
      PointState<TP> s;
      const uint32_t code = propagate_point<TS, TP, kVec>(rv, int64_t(sat), g, t[j], s);
      out.put(int64_t(sat) * T + j, code, s);
    }
  }
}

// ------------------------------------------------------------ ragged tiles --
// tile_start[w]: first point of tile w; tile_meta[2w], tile_meta[2w + 1]: its
// satellite and its length (<= 64 points of that satellite's list).
//
// tile_once_kernel: the grid covers every tile, one wavefront each and no
// loop, like the dense kernel: the wavefront ends after its stores, so nothing
// waits for them.  tiles_kernel: a persistent grid whose wavefronts loop over
// tiles (fewer workgroups; each iteration waits for the previous one's stores
// before reusing their registers).
template <class TS, class TP, int kBlock, bool kOff32, bool kDeep>
__global__ void __launch_bounds__(kBlock) SGP4MI_TILE_OCCUPANCY tile_once_kernel(RecordView rv, const double* __restrict__ t,
                                                           const int64_t* __restrict__ tile_start,
                                                           const int32_t* __restrict__ tile_meta, int64_t ntiles,
                                                           Out<TP, kOff32> out) {
  constexpr int kWaves = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int64_t w = int64_t(blockIdx.x) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= ntiles) return;
  const int64_t start = tile_start[w];
  const int32_t sat = tile_meta[2 * w];
  const int32_t len = tile_meta[2 * w + 1];
  if (lane >= len) return;
  const Grav g = load_grav(rv);
  const int64_t p = kOff32 ? int64_t(uint32_t(start) + uint32_t(lane)) : start + lane;  // kOff32: p < 2^30
  PointState<TP> s;
  const uint32_t code = propagate_point<TS, TP, false, kDeep>(rv, sat, g, t[p], s);
  out.put(p, code, s);
}

template <class TS, class TP, int kBlock, bool kOff32, bool kDeep>
__global__ void __launch_bounds__(kBlock) tiles_kernel(RecordView rv, const double* __restrict__ t,
                                                       const int64_t* __restrict__ tile_start,
                                                       const int32_t* __restrict__ tile_meta, int64_t ntiles,
                                                       Out<TP, kOff32> out) {
  constexpr int kWaves = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = int64_t(blockIdx.x) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = int64_t(gridDim.x) * kWaves;
  const Grav g = load_grav(rv);
  for (int64_t w = wave0; w < ntiles; w += nwaves) {
    const int64_t start = tile_start[w];
    const int32_t sat = __builtin_amdgcn_readfirstlane(tile_meta[2 * w]);
    const int32_t len = __builtin_amdgcn_readfirstlane(tile_meta[2 * w + 1]);
    if (lane < len) {
      PointState<TP> s;  // satellite uniform: scalar constants
      const uint32_t code = propagate_point<TS, TP, false, kDeep>(rv, sat, g, t[start + lane], s);
      out.put(start + lane, code, s);
    }
  }
}

// ------------------------------------------------------------- ragged flat --
// chunk_sat[k]: satellite whose list contains point 64*k.  When chunk_sat is
// null the wavefront finds it by a 64-way search of the offsets (each round
// every lane probes one of 64 evenly spaced offsets of [lo, hi) and a ballot
// keeps the piece holding q).  The offsets are then unchecked caller data: the
// search and the walk read only offsets[0..n] and yield a satellite in [0, n)
// whatever they hold, and a point outside that satellite's list (possible only
// for malformed offsets) gets code 8 and NaN instead of a state.
template <class TS, class TP, int kBlock, bool kOff32>
__global__ void __launch_bounds__(kBlock) flat_kernel(RecordView rv, const int64_t* __restrict__ offsets, int64_t n,
                                                      const double* __restrict__ t, int64_t nnz,
                                                      const int32_t* __restrict__ chunk_sat, int64_t nchunks,
                                                      Out<TP, kOff32> out) {
  constexpr int kWaves = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = int64_t(blockIdx.x) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = int64_t(gridDim.x) * kWaves;
  const Grav g = load_grav(rv);
  for (int64_t k = wave0; k < nchunks; k += nwaves) {
    const int64_t q = k * 64;
    const int64_t first = chunk_sat ? int64_t(chunk_sat[k])
                                    : wave_search(n, [&](int64_t lo, int64_t step, int64_t hi) {
                                        const int64_t idx = lo + step * lane;
                                        return uint64_t(__ballot(idx < hi && offsets[idx] <= q));
                                      });
    const int64_t p = q + lane;
    if (p < nnz) {
      bool owned;
      const int64_t sat = point_owner(offsets, n, first, p, &owned);
      PointState<TP> s;
      s.ok = false;
      uint32_t code = kCodeUnowned;
      if (owned) {
        code = propagate_point<TS, TP, true>(rv, sat, g, t[p], s);
      }
      out.put(p, code, s);
    }
  }
}

// ------------------------------------------------------------- launchers --
template <class TP>
static bool fits32(int64_t P) {
  return P >= 0 && uint64_t(P) * sizeof(TP) < (uint64_t(1) << 32);
}

template <class TS, class TP, int kBlock, bool kVec, bool kOff32>
static void dense_go(dim3 grid, hipStream_t s, const RecordView& rv, const double* t, int64_t T, void* r, void* v,
                     uint8_t* err, int64_t P) {
  Out<TP, kOff32> o{static_cast<TP*>(r), static_cast<TP*>(v), err, P};
  if (int64_t(grid.y) * kBlock >= T)
    hipLaunchKernelGGL((dense_kernel<TS, TP, kBlock, kVec, kOff32, false>), grid, dim3(kBlock), 0, s, rv, t, T, o);
  else
    hipLaunchKernelGGL((dense_kernel<TS, TP, kBlock, kVec, kOff32, true>), grid, dim3(kBlock), 0, s, rv, t, T, o);
}

template <class TS, class TP, int kBlock>
static void dense_b(dim3 grid, hipStream_t s, bool vec, const RecordView& rv, const double* t, int64_t T, void* r,
                    void* v, uint8_t* err, int64_t P) {
  const bool o32 = fits32<TP>(P);
  if (vec) {
    if (o32) dense_go<TS, TP, kBlock, true, true>(grid, s, rv, t, T, r, v, err, P);
    else dense_go<TS, TP, kBlock, true, false>(grid, s, rv, t, T, r, v, err, P);
  } else {
    if (o32) dense_go<TS, TP, kBlock, false, true>(grid, s, rv, t, T, r, v, err, P);
    else dense_go<TS, TP, kBlock, false, false>(grid, s, rv, t, T, r, v, err, P);
  }
}

template <class TS, class TP>
static hipError_t dense_t(const RecordView& rv, int64_t n, const double* t, int64_t T, void* r, void* v,
                          uint8_t* err, int block, bool vec, hipStream_t s) {
  const int64_t tiles = (T + block - 1) / block;
  const unsigned gy = unsigned(tiles < 65535 ? tiles : 65535);
  const dim3 grid(unsigned(n), gy);
  const int64_t P = n * T;
  switch (block) {
    case 64: dense_b<TS, TP, 64>(grid, s, vec, rv, t, T, r, v, err, P); break;
    case 128: dense_b<TS, TP, 128>(grid, s, vec, rv, t, T, r, v, err, P); break;
    case 256: dense_b<TS, TP, 256>(grid, s, vec, rv, t, T, r, v, err, P); break;
    case 512: dense_b<TS, TP, 512>(grid, s, vec, rv, t, T, r, v, err, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class TS, class TP, int kBlock, bool kVec>
static void persist_go(unsigned grid, hipStream_t s, const RecordView& rv, const double* t, int64_t T, int64_t n,
                       void* r, void* v, uint8_t* err) {
  const int64_t P = n * T;
  const uint32_t tps = uint32_t((T + 63) / 64);
  const uint64_t ntiles = uint64_t(n) * tps;
  if (fits32<TP>(P)) {
    Out<TP, true> o{static_cast<TP*>(r), static_cast<TP*>(v), err, P};
    hipLaunchKernelGGL((dense_persistent_kernel<TS, TP, kBlock, kVec, true>), dim3(grid), dim3(kBlock), 0, s, rv, t,
                       T, tps, ntiles, o);
  } else {
    Out<TP, false> o{static_cast<TP*>(r), static_cast<TP*>(v), err, P};
    hipLaunchKernelGGL((dense_persistent_kernel<TS, TP, kBlock, kVec, false>), dim3(grid), dim3(kBlock), 0, s, rv, t,
                       T, tps, ntiles, o);
  }
}

template <class TS, class TP>
static hipError_t persist_t(const RecordView& rv, int64_t n, const double* t, int64_t T, void* r, void* v,
                            uint8_t* err, int block, bool vec, unsigned grid, hipStream_t s) {
#define SGP4MI_PERSIST(B)                                                       \
  if (vec) persist_go<TS, TP, B, true>(grid, s, rv, t, T, n, r, v, err);        \
  else persist_go<TS, TP, B, false>(grid, s, rv, t, T, n, r, v, err);
  switch (block) {
    case 64: SGP4MI_PERSIST(64) break;
    case 128: SGP4MI_PERSIST(128) break;
    case 256: SGP4MI_PERSIST(256) break;
    case 512: SGP4MI_PERSIST(512) break;
    default: return hipErrorInvalidValue;
  }
#undef SGP4MI_PERSIST
  return hipGetLastError();
}

template <class TS, class TP, int kBlock>
static void tile_go(hipStream_t s, const RecordView& rv, const double* t, int64_t T, int64_t n, void* r, void* v,
                    uint8_t* err) {
  const int64_t P = n * T;
  const uint32_t tps = uint32_t((T + 63) / 64);
  const uint32_t ntiles = uint32_t(n * tps);
  const unsigned grid = unsigned((int64_t(ntiles) + kBlock / 64 - 1) / (kBlock / 64));
  if (fits32<TP>(P)) {
    Out<TP, true> o{static_cast<TP*>(r), static_cast<TP*>(v), err, P};
    hipLaunchKernelGGL((dense_tile_kernel<TS, TP, kBlock, true>), dim3(grid), dim3(kBlock), 0, s, rv, t, T, tps,
                       ntiles, o);
  } else {
    Out<TP, false> o{static_cast<TP*>(r), static_cast<TP*>(v), err, P};
    hipLaunchKernelGGL((dense_tile_kernel<TS, TP, kBlock, false>), dim3(grid), dim3(kBlock), 0, s, rv, t, T, tps,
                       ntiles, o);
  }
}

template <class TS, class TP>
static hipError_t tile_t(const RecordView& rv, int64_t n, const double* t, int64_t T, void* r, void* v, uint8_t* err,
                         int block, hipStream_t s) {
  switch (block) {
    case 64: tile_go<TS, TP, 64>(s, rv, t, T, n, r, v, err); break;
    case 128: tile_go<TS, TP, 128>(s, rv, t, T, n, r, v, err); break;
    case 256: tile_go<TS, TP, 256>(s, rv, t, T, n, r, v, err); break;
    case 512: tile_go<TS, TP, 512>(s, rv, t, T, n, r, v, err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class TS, class TP, int kBlock>
static void flat_go(hipStream_t s, const RecordView& rv, const double* t, int64_t T, int64_t n, void* r, void* v,
                    uint8_t* err) {
  const int64_t P = n * T;
  const unsigned grid = unsigned((P + kBlock - 1) / kBlock);
  if (fits32<TP>(P)) {
    Out<TP, true> o{static_cast<TP*>(r), static_cast<TP*>(v), err, P};
    hipLaunchKernelGGL((dense_flat_kernel<TS, TP, kBlock, true>), dim3(grid), dim3(kBlock), 0, s, rv, t, T, o);
  } else {
    Out<TP, false> o{static_cast<TP*>(r), static_cast<TP*>(v), err, P};
    hipLaunchKernelGGL((dense_flat_kernel<TS, TP, kBlock, false>), dim3(grid), dim3(kBlock), 0, s, rv, t, T, o);
  }
}

template <class TS, class TP>
static hipError_t flat_t(const RecordView& rv, int64_t n, const double* t, int64_t T, void* r, void* v, uint8_t* err,
                         int block, hipStream_t s) {
  switch (block) {
    case 64: flat_go<TS, TP, 64>(s, rv, t, T, n, r, v, err); break;
    case 128: flat_go<TS, TP, 128>(s, rv, t, T, n, r, v, err); break;
    case 256: flat_go<TS, TP, 256>(s, rv, t, T, n, r, v, err); break;
    case 512: flat_go<TS, TP, 512>(s, rv, t, T, n, r, v, err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Whether the flat dense grid (one lane per point, ceil(n T / block)
// workgroups) fits the launch limits: fewer than 2^31 workgroups and 2^32
// work-items.
bool dense_flat_fits(int64_t n, int64_t T, int block) {
  const int64_t groups = (n * T + block - 1) / block;
  return groups <= int64_t(0x7fffffff) && grid_fits(uint64_t(groups), uint64_t(block));
}

// Whether the one-wavefront-per-64-time-tile grid of an n x T batch fits:
// 32-bit tile indices, and ceil(tiles / (block / 64)) workgroups of block
// lanes within the 2^32 work-item extent of a dispatch.
bool dense_tiles_fit(int64_t n, int64_t T, int block) {
  const int64_t tps = (T + 63) / 64;
  if (!(n <= INT64_MAX / (tps > 0 ? tps : 1) && n * tps <= 0xffffffffLL)) return false;
  const int64_t groups = (n * tps + block / 64 - 1) / (block / 64);
  return grid_fits(uint64_t(groups), uint64_t(block));
}

// Whether the satellite-by-time grid (n workgroups in x) fits.
bool dense_grid_fits(int64_t n, int block) { return grid_fits(uint64_t(n), uint64_t(block)); }

// block: workgroup size; vec: constants through vector loads (else scalar);
// grid > 0 selects the persistent kernel with that many workgroups; tiles
// selects one wavefront per 64-time tile (scalar constants; the caller checks
// dense_tiles_fit); flat one lane per point in point order (vector constants;
// the caller checks dense_flat_fits).
hipError_t launch_dense(int precision, const void* consts, int64_t n, const double* t, int64_t T, void* r, void* v,
                        uint8_t* err, int block, bool vec, unsigned grid, bool tiles, bool flat, hipStream_t s) {
  const RecordView rv = view_of(consts, n);
  if (flat) {
    switch (precision) {
      case 0: return flat_t<double, double>(rv, n, t, T, r, v, err, block, s);
      case 1: return flat_t<float, float>(rv, n, t, T, r, v, err, block, s);
      case 2: return flat_t<double, float>(rv, n, t, T, r, v, err, block, s);
    }
    return hipErrorInvalidValue;
  }
  if (tiles) {
    switch (precision) {
      case 0: return tile_t<double, double>(rv, n, t, T, r, v, err, block, s);
      case 1: return tile_t<float, float>(rv, n, t, T, r, v, err, block, s);
      case 2: return tile_t<double, float>(rv, n, t, T, r, v, err, block, s);
    }
    return hipErrorInvalidValue;
  }
  if (grid > 0) {
    switch (precision) {
      case 0: return persist_t<double, double>(rv, n, t, T, r, v, err, block, vec, grid, s);
      case 1: return persist_t<float, float>(rv, n, t, T, r, v, err, block, vec, grid, s);
      case 2: return persist_t<double, float>(rv, n, t, T, r, v, err, block, vec, grid, s);
    }
    return hipErrorInvalidValue;
  }
  switch (precision) {
    case 0: return dense_t<double, double>(rv, n, t, T, r, v, err, block, vec, s);
    case 1: return dense_t<float, float>(rv, n, t, T, r, v, err, block, vec, s);
    case 2: return dense_t<double, float>(rv, n, t, T, r, v, err, block, vec, s);
  }
  return hipErrorInvalidValue;
}

template <class TS, class TP, int kBlock, bool kOff32>
static void ragged_go(int mode, bool deep, unsigned grid, hipStream_t s, const RecordView& rv,
                      const int64_t* offsets, int64_t n, const double* t, int64_t nnz, const int64_t* tile_start,
                      const int32_t* tile_sat, int64_t ntiles, void* r, void* v, uint8_t* err) {
  Out<TP, kOff32> o{static_cast<TP*>(r), static_cast<TP*>(v), err, nnz};
  if (mode == 0 && int64_t(grid) * (kBlock / 64) >= ntiles) {
    if (deep)
      hipLaunchKernelGGL((tile_once_kernel<TS, TP, kBlock, kOff32, true>), dim3(grid), dim3(kBlock), 0, s, rv, t,
                         tile_start, tile_sat, ntiles, o);
    else
      hipLaunchKernelGGL((tile_once_kernel<TS, TP, kBlock, kOff32, false>), dim3(grid), dim3(kBlock), 0, s, rv, t,
                         tile_start, tile_sat, ntiles, o);
  } else if (mode == 0) {
    if (deep)
      hipLaunchKernelGGL((tiles_kernel<TS, TP, kBlock, kOff32, true>), dim3(grid), dim3(kBlock), 0, s, rv, t,
                         tile_start, tile_sat, ntiles, o);
    else
      hipLaunchKernelGGL((tiles_kernel<TS, TP, kBlock, kOff32, false>), dim3(grid), dim3(kBlock), 0, s, rv, t,
                         tile_start, tile_sat, ntiles, o);
  }
  else
    hipLaunchKernelGGL((flat_kernel<TS, TP, kBlock, kOff32>), dim3(grid), dim3(kBlock), 0, s, rv, offsets, n, t, nnz,
                       tile_sat, ntiles, o);
}

template <class TS, class TP, int kBlock>
static void ragged_b(int mode, bool deep, unsigned grid, hipStream_t s, const RecordView& rv, const int64_t* offsets,
                     int64_t n, const double* t, int64_t nnz, const int64_t* tile_start, const int32_t* tile_sat,
                     int64_t ntiles, void* r, void* v, uint8_t* err) {
  if (fits32<TP>(nnz))
    ragged_go<TS, TP, kBlock, true>(mode, deep, grid, s, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v,
                                    err);
  else
    ragged_go<TS, TP, kBlock, false>(mode, deep, grid, s, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v,
                                     err);
}

template <class TS, class TP>
static hipError_t ragged_t(int mode, bool deep, const RecordView& rv, const int64_t* offsets, int64_t n,
                           const double* t, int64_t nnz, const int64_t* tile_start, const int32_t* tile_sat,
                           int64_t ntiles, void* r, void* v, uint8_t* err, int block, unsigned grid, hipStream_t s) {
  switch (block) {
    case 64: ragged_b<TS, TP, 64>(mode, deep, grid, s, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v, err); break;
    case 128: ragged_b<TS, TP, 128>(mode, deep, grid, s, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v, err); break;
    case 256: ragged_b<TS, TP, 256>(mode, deep, grid, s, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v, err); break;
    case 512: ragged_b<TS, TP, 512>(mode, deep, grid, s, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v, err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// mode 0: tiles (tile_start and the (satellite, length) pairs in tile_sat, of
// ntiles tiles; one wavefront per tile when the grid covers them all, else a
// persistent loop); mode 1: flat (tile_sat holds
// the chunk satellites of ntiles = ceil(nnz / 64) chunks or is null for the
// in-kernel search; tile_start unused).  deep = false (mode 0 only): the
// record holds no deep-space satellite; kernels without the deep-space branch.
hipError_t launch_ragged(int precision, int mode, bool deep, const void* consts, int64_t n, const int64_t* offsets,
                         const double* t, int64_t nnz, const int64_t* tile_start, const int32_t* tile_sat,
                         int64_t ntiles, void* r, void* v, uint8_t* err, int block, unsigned grid, hipStream_t s) {
  const RecordView rv = view_of(consts, n);
  deep = deep || mode != 0;
  switch (precision) {
    case 0: return ragged_t<double, double>(mode, deep, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v,
                                            err, block, grid, s);
    case 1: return ragged_t<float, float>(mode, deep, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v,
                                          err, block, grid, s);
    case 2: return ragged_t<double, float>(mode, deep, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v,
                                           err, block, grid, s);
  }
  return hipErrorInvalidValue;
}

// Whether any satellite of the record carries the deep-space bit: *flag (a
// device word) is cleared, then set by every lane whose satellite has it.
__global__ void clear_word_kernel(uint32_t* flag) { *flag = 0u; }
__global__ void __launch_bounds__(256) any_deep_kernel(RecordView rv, int64_t n, uint32_t* flag) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n && (rv.slots[i].info & kInfoDeep)) atomicOr(flag, 1u);
}
hipError_t launch_any_deep(const void* consts, int64_t n, uint32_t* flag, hipStream_t s) {
  const RecordView rv = view_of(consts, n);
  hipLaunchKernelGGL(clear_word_kernel, dim3(1), dim3(1), 0, s, flag);
  const int64_t blocks = (n + 255) / 256;
  // the grid in chunks of at most 2^31 - 1 workgroups is never needed: n < 2^31 here
  hipLaunchKernelGGL(any_deep_kernel, dim3(unsigned(blocks > 0 ? blocks : 1)), dim3(256), 0, s, rv, n, flag);
  return hipGetLastError();
}

}  // namespace sgp4mi

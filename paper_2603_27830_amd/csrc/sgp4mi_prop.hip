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
// Outputs are component-major SoA, r[c * P + p], written with non-temporal
// stores; codes 1, 2, 4 and 7 write NaN states.
#include "sgp4mi_point.h"

namespace sgp4mi {

template <class TP>
__device__ __forceinline__ void store_point(TP* __restrict__ r, TP* __restrict__ v, uint8_t* __restrict__ err,
                                            int64_t P, int64_t p, uint32_t code, const PointState<TP>& s) {
  TP x0 = s.r[0], x1 = s.r[1], x2 = s.r[2], y0 = s.v[0], y1 = s.v[1], y2 = s.v[2];
  if (code != 0 && code != 6) {
    const TP q = TP(__builtin_nan(""));
    x0 = x1 = x2 = y0 = y1 = y2 = q;
  }
  st_nt(r + p, x0);
  st_nt(r + P + p, x1);
  st_nt(r + 2 * P + p, x2);
  st_nt(v + p, y0);
  st_nt(v + P + p, y1);
  st_nt(v + 2 * P + p, y2);
  st_nt(err + p, uint8_t(code));
}

// ------------------------------------------------------------------ dense --
template <class TS, class TP, int kBlock>
__global__ void __launch_bounds__(kBlock) dense_kernel(RecordView rv, const double* __restrict__ t, int64_t T,
                                                       TP* __restrict__ r, TP* __restrict__ v,
                                                       uint8_t* __restrict__ err, int64_t P) {
  const int64_t i = blockIdx.x;
  const SatC<TS, TP> c = load_sat<TS, TP>(rv, i);
  const Grav g = load_grav(rv);
  for (int64_t j = int64_t(blockIdx.y) * kBlock + threadIdx.x; j < T; j += int64_t(gridDim.y) * kBlock) {
    PointState<TP> s;
    const uint32_t code = sgp4_point<TS, TP>(c, g, t[j], s);
    store_point(r, v, err, P, i * T + j, code, s);
  }
}

// ------------------------------------------------------------ ragged tiles --
// tile_start[w]: first point of tile w; tile_sat[w]: its satellite.  A tile
// holds min(64, end of that satellite's list - tile_start) points.
template <class TS, class TP, int kBlock>
__global__ void __launch_bounds__(kBlock) tiles_kernel(RecordView rv, const int64_t* __restrict__ offsets,
                                                       const double* __restrict__ t, int64_t nnz,
                                                       const int64_t* __restrict__ tile_start,
                                                       const int32_t* __restrict__ tile_sat, int64_t ntiles,
                                                       TP* __restrict__ r, TP* __restrict__ v,
                                                       uint8_t* __restrict__ err) {
  constexpr int kWaves = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = int64_t(blockIdx.x) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = int64_t(gridDim.x) * kWaves;
  const Grav g = load_grav(rv);
  for (int64_t w = wave0; w < ntiles; w += nwaves) {
    const int64_t start = tile_start[w];
    const int32_t sat = __builtin_amdgcn_readfirstlane(tile_sat[w]);
    const int64_t end = offsets[sat + 1];
    const SatC<TS, TP> c = load_sat<TS, TP>(rv, sat);
    const int64_t p = start + lane;
    if (p < end && p - start < 64) {
      PointState<TP> s;
      const uint32_t code = sgp4_point<TS, TP>(c, g, t[p], s);
      store_point(r, v, err, nnz, p, code, s);
    }
  }
}

// ------------------------------------------------------------- ragged flat --
// chunk_sat[k]: satellite whose list contains point 64*k.  When chunk_sat is
// null the wavefront finds it by a uniform binary search of the offsets.
template <class TS, class TP, int kBlock>
__global__ void __launch_bounds__(kBlock) flat_kernel(RecordView rv, const int64_t* __restrict__ offsets, int64_t n,
                                                      const double* __restrict__ t, int64_t nnz,
                                                      const int32_t* __restrict__ chunk_sat, int64_t nchunks,
                                                      TP* __restrict__ r, TP* __restrict__ v,
                                                      uint8_t* __restrict__ err) {
  constexpr int kWaves = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = int64_t(blockIdx.x) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = int64_t(gridDim.x) * kWaves;
  const Grav g = load_grav(rv);
  for (int64_t k = wave0; k < nchunks; k += nwaves) {
    int64_t first;
    if (chunk_sat) {
      first = chunk_sat[k];
    } else {
      // offsets[lo] <= q < offsets[hi] holds throughout (offsets[0] = 0 <= q < nnz = offsets[n]).
      const int64_t q = k * 64;
      int64_t lo = 0, hi = n;
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (offsets[mid] <= q) lo = mid; else hi = mid;
      }
      first = lo;
    }
    const int64_t p = k * 64 + lane;
    if (p < nnz) {
      int64_t sat = first;
      while (sat + 1 < n && offsets[sat + 1] <= p) ++sat;
      const SatC<TS, TP> c = load_sat<TS, TP>(rv, sat);
      PointState<TP> s;
      const uint32_t code = sgp4_point<TS, TP>(c, g, t[p], s);
      store_point(r, v, err, nnz, p, code, s);
    }
  }
}

// ------------------------------------------------------------- launchers --
template <class TS, class TP>
static hipError_t dense_t(const RecordView& rv, int64_t n, const double* t, int64_t T, void* r, void* v,
                          uint8_t* err, int block, hipStream_t s) {
  const int64_t tiles = (T + block - 1) / block;
  const unsigned gy = unsigned(tiles < 65535 ? tiles : 65535);
  const dim3 grid(unsigned(n), gy);
  TP* rr = static_cast<TP*>(r);
  TP* vv = static_cast<TP*>(v);
  const int64_t P = n * T;
  switch (block) {
    case 64: hipLaunchKernelGGL((dense_kernel<TS, TP, 64>), grid, dim3(64), 0, s, rv, t, T, rr, vv, err, P); break;
    case 128: hipLaunchKernelGGL((dense_kernel<TS, TP, 128>), grid, dim3(128), 0, s, rv, t, T, rr, vv, err, P); break;
    case 256: hipLaunchKernelGGL((dense_kernel<TS, TP, 256>), grid, dim3(256), 0, s, rv, t, T, rr, vv, err, P); break;
    case 512: hipLaunchKernelGGL((dense_kernel<TS, TP, 512>), grid, dim3(512), 0, s, rv, t, T, rr, vv, err, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dense(int precision, const void* consts, int64_t n, const double* t, int64_t T, void* r, void* v,
                        uint8_t* err, int block, hipStream_t s) {
  const RecordView rv = view_of(consts, n);
  switch (precision) {
    case 0: return dense_t<double, double>(rv, n, t, T, r, v, err, block, s);
    case 1: return dense_t<float, float>(rv, n, t, T, r, v, err, block, s);
    case 2: return dense_t<double, float>(rv, n, t, T, r, v, err, block, s);
  }
  return hipErrorInvalidValue;
}

template <class TS, class TP, int kBlock>
static void tiles_t(const RecordView& rv, const int64_t* offsets, const double* t, int64_t nnz,
                    const int64_t* tile_start, const int32_t* tile_sat, int64_t ntiles, void* r, void* v,
                    uint8_t* err, unsigned grid, hipStream_t s) {
  hipLaunchKernelGGL((tiles_kernel<TS, TP, kBlock>), dim3(grid), dim3(kBlock), 0, s, rv, offsets, t, nnz, tile_start,
                     tile_sat, ntiles, static_cast<TP*>(r), static_cast<TP*>(v), err);
}

template <class TS, class TP, int kBlock>
static void flat_t(const RecordView& rv, const int64_t* offsets, int64_t n, const double* t, int64_t nnz,
                   const int32_t* chunk_sat, int64_t nchunks, void* r, void* v, uint8_t* err, unsigned grid,
                   hipStream_t s) {
  hipLaunchKernelGGL((flat_kernel<TS, TP, kBlock>), dim3(grid), dim3(kBlock), 0, s, rv, offsets, n, t, nnz, chunk_sat,
                     nchunks, static_cast<TP*>(r), static_cast<TP*>(v), err);
}

#define SGP4MI_BLOCKS(F, ...)                               \
  switch (block) {                                          \
    case 64: F<TS, TP, 64>(__VA_ARGS__); break;             \
    case 128: F<TS, TP, 128>(__VA_ARGS__); break;           \
    case 256: F<TS, TP, 256>(__VA_ARGS__); break;           \
    case 512: F<TS, TP, 512>(__VA_ARGS__); break;           \
    default: return hipErrorInvalidValue;                   \
  }

template <class TS, class TP>
static hipError_t ragged_t(int mode, const RecordView& rv, const int64_t* offsets, int64_t n, const double* t,
                           int64_t nnz, const int64_t* tile_start, const int32_t* tile_sat, int64_t ntiles, void* r,
                           void* v, uint8_t* err, int block, unsigned grid, hipStream_t s) {
  if (mode == 0) {
    SGP4MI_BLOCKS(tiles_t, rv, offsets, t, nnz, tile_start, tile_sat, ntiles, r, v, err, grid, s)
  } else {
    SGP4MI_BLOCKS(flat_t, rv, offsets, n, t, nnz, tile_sat, ntiles, r, v, err, grid, s)
  }
  return hipGetLastError();
}

// mode 0: tiles (tile_start/tile_sat of ntiles); mode 1: flat (tile_sat holds
// the chunk satellites of ntiles = ceil(nnz / 64) chunks, tile_start unused).
hipError_t launch_ragged(int precision, int mode, const void* consts, int64_t n, const int64_t* offsets,
                         const double* t, int64_t nnz, const int64_t* tile_start, const int32_t* tile_sat,
                         int64_t ntiles, void* r, void* v, uint8_t* err, int block, unsigned grid, hipStream_t s) {
  const RecordView rv = view_of(consts, n);
  switch (precision) {
    case 0: return ragged_t<double, double>(mode, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v, err,
                                            block, grid, s);
    case 1: return ragged_t<float, float>(mode, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v, err,
                                          block, grid, s);
    case 2: return ragged_t<double, float>(mode, rv, offsets, n, t, nnz, tile_start, tile_sat, ntiles, r, v, err,
                                           block, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace sgp4mi

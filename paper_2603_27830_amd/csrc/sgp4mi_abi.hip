// C ABI of the library: argument validation, launch selection, ragged plans
// (tile tables, autotuner, HIP graph capture).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "sgp4mi.h"
#include "sgp4mi_common.h"

namespace sgp4mi {
hipError_t launch_init(const double g[5], double ref_day, int64_t n, const double* elem, void* consts,
                       uint8_t* user_flags, hipStream_t s);
hipError_t launch_dense(int precision, const void* consts, int64_t n, const double* t, int64_t T, void* r, void* v,
                        uint8_t* err, int block, bool vec, unsigned grid, bool tiles, bool flat, hipStream_t s);
bool dense_tiles_fit(int64_t n, int64_t T, int block);
bool dense_grid_fits(int64_t n, int block);
bool fused_fits(int64_t n, int64_t T);
bool dense_flat_fits(int64_t n, int64_t T, int block);
hipError_t launch_fused(int precision, const double g[5], double ref_day, int64_t n, const double* elem,
                        const double* t, int64_t T, void* r, void* v, uint8_t* err, uint8_t* user_flags,
                        hipStream_t s);
int64_t fused_max_T();
hipError_t launch_screen(const void* r, bool fp64, const uint8_t* err, int64_t n, int64_t T, double D, int64_t cap,
                         int32_t* pairs, double* dist, unsigned long long* count, void* ws, int mode, hipStream_t s);
int screen_max_n();
size_t screen_ws_bytes(int64_t n, int64_t T);
bool screen_global_fits(int64_t n, int64_t T);
size_t screen_static_bytes();
hipError_t launch_screen_static(const void* r, bool fp64, const uint8_t* err, int64_t n, int64_t T, double D,
                                int64_t cap, int32_t* pairs, double* dist, unsigned long long* count, hipStream_t s);
hipError_t launch_ragged(int precision, int mode, bool deep, const void* consts, int64_t n, const int64_t* offsets,
                         const double* t, int64_t nnz, const int64_t* tile_start, const int32_t* tile_sat,
                         int64_t ntiles, void* r, void* v, uint8_t* err, int block, unsigned grid, hipStream_t s);
hipError_t launch_any_deep(const void* consts, int64_t n, uint32_t* flag, hipStream_t s);
hipError_t launch_vjp(int precision, int64_t n, const double* elem, const void* consts, const double* t, int64_t T,
                      const void* gr, const void* gv, double* gelem, hipStream_t s);
hipError_t launch_vjp_ragged(int precision, int64_t n, const double* elem, const void* consts, const int64_t* offsets,
                             const double* t, int64_t nnz, const void* gr, const void* gv, double* gelem,
                             hipStream_t s);
hipError_t launch_jacobian_ragged(int precision, int64_t n, const double* elem, const void* consts,
                                  const int64_t* offsets, const double* t, int64_t nnz, double* jac, hipStream_t s);
hipError_t launch_jacobian(int precision, int64_t n, const double* elem, const void* consts, const double* t,
                           int64_t T, double* jac, hipStream_t s);
}  // namespace sgp4mi

using namespace sgp4mi;

namespace {

constexpr double kWgs72[5] = {398600.8, 6378.135, 0.001082616, -0.00000253881, -0.00000165597};
constexpr int64_t kMaxSats = 2147483647LL;
// Time lists shorter than this take the flat dense mapping (one lane per
// point in point order) instead of 64-time tiles, most of whose lanes would
// be idle.
constexpr int64_t kFlatBelowT = 64;
// Elements-to-states calls with at most this many times run the fused
// kernel (initialisation kept on chip); longer ones, given a record
// workspace, run initialisation and the default dense launch.
constexpr int64_t kFusedMaxT = 32;
// Workgroup size of the VJP and Jacobian kernels (one workgroup per satellite).
constexpr uint64_t kVjpLanes = 256;
// Default dense launch: one wavefront per 64-time tile with the satellite's
// constants in scalar registers, in 256-wide workgroups for FP64 and 512-wide
// for the float paths (fastest of the mapping x workgroup x residency sweep on
// MI355X at 9,341 x 1,000); the satellite-by-time grid where the tiles do not
// fit the launch limits, and beyond that a persistent grid of 512-wide
// workgroups (four per compute unit) looping over the tiles.
int default_dense(int precision, int64_t n, int64_t T) {
  if (T < kFlatBelowT && dense_flat_fits(n, T, 256)) return 256 | SGP4_CFG_FLAT;
  const int block = precision == SGP4_FP64 ? 256 : 512;
  if (!dense_tiles_fit(n, T, block)) return 512 | SGP4_CFG_SCALAR_CONSTS | SGP4_CFG_PERSISTENT | SGP4_CFG_PER_CU(4);
  return block | SGP4_CFG_SCALAR_CONSTS | SGP4_CFG_TILES;
}

// Reference instant of the epoch row (host {whole, frac} Julian date, NULL =
// J2000.0) as days after JD 2415020.0, the origin of the lunar and solar
// arguments of the deep-space terms; false when not finite.
bool ref_day_of(const double* ref_jd, double* day) {
  const double w = ref_jd ? ref_jd[0] : 2451545.0, f = ref_jd ? ref_jd[1] : 0.0;
  *day = (w - 2415020.0) + f;
  return std::isfinite(*day);
}

int check_gravity(const double* g) {
  for (int k = 0; k < 5; ++k)
    if (!std::isfinite(g[k])) return SGP4_E_GRAVITY;
  if (!(g[0] > 0) || !(g[1] > 0)) return SGP4_E_GRAVITY;
  if (g[2] == 0.0 && g[3] != 0.0) return SGP4_E_GRAVITY;
  return SGP4_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? SGP4_OK : SGP4_E_HIP; }

bool mul_overflows(int64_t a, int64_t b) { return a != 0 && b > INT64_MAX / a; }

int compute_units() {
  static int cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  });
  return cus;
}

}  // namespace

// ------------------------------------------------------------------- plans --
struct sgp4_plan {
  int precision = 0;
  int mode = 1;      // 0 tiles, 1 flat
  int block = 256;
  unsigned grid = 0;
  const void* consts = nullptr;
  int64_t n = 0, nnz = 0;
  const int64_t* offsets = nullptr;
  const double* t = nullptr;
  void* r = nullptr;
  void* v = nullptr;
  uint8_t* err = nullptr;
  int64_t* tile_start = nullptr;  // device, tiles mode
  int32_t* tile_sat = nullptr;    // device, tiles mode: (satellite, length) pairs
  int64_t ntiles = 0;
  int32_t* chunk_sat = nullptr;   // device, flat mode
  int64_t nchunks = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // whether the record held a deep-space satellite when the plan was made;
  // without one the tile kernels are the ones compiled without that branch
  bool deep = true;
  double best_us = -1.0;
  int ncandidates = 0;
  bool from_cache = false;
};

namespace {

hipError_t plan_launch_direct(const sgp4_plan* p, hipStream_t s) {
  if (p->mode == 0)
    return launch_ragged(p->precision, 0, p->deep, p->consts, p->n, p->offsets, p->t, p->nnz, p->tile_start,
                         p->tile_sat, p->ntiles, p->r, p->v, p->err, p->block, p->grid, s);
  return launch_ragged(p->precision, 1, true, p->consts, p->n, p->offsets, p->t, p->nnz, nullptr, p->chunk_sat,
                       p->nchunks, p->r, p->v, p->err, p->block, p->grid, s);
}

void plan_free(sgp4_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->tile_start) (void)hipFree(p->tile_start);
  if (p->tile_sat) (void)hipFree(p->tile_sat);
  if (p->chunk_sat) (void)hipFree(p->chunk_sat);
  delete p;
}

// Tuning cache: one line per key, "key mode block grid us".
std::string cache_path() {
  const char* e = std::getenv("SGP4MI_TUNE_CACHE");
  if (e && *e) return e;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/sgp4mi_tune.txt";
}

std::string tune_key(const sgp4_plan* p) {
  // Keyed by device, precision, whether the record holds deep-space
  // satellites and the batch's size class (powers of two of n and nnz): a
  // plan for a similar batch reuses the choice.
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  for (auto& ch : arch) if (ch == ' ' || ch == ':') ch = '_';
  char buf[256];
  std::snprintf(buf, sizeof buf, "v4/%s/p%d/d%d/n%d/z%d", arch.c_str(), p->precision, p->deep ? 1 : 0,
                int(std::log2(double(p->n) + 1)), int(std::log2(double(p->nnz) + 1)));
  return buf;
}

bool cache_lookup(const std::string& key, int* mode, int* block, unsigned* grid, double* us) {
  FILE* f = std::fopen(cache_path().c_str(), "r");
  if (!f) return false;
  char k[200];
  int m, b;
  unsigned g;
  double u;
  bool found = false;
  while (std::fscanf(f, "%199s %d %d %u %lf", k, &m, &b, &g, &u) == 5) {
    if (key == k) { *mode = m; *block = b; *grid = g; *us = u; found = true; }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& key, int mode, int block, unsigned grid, double us) {
  std::string path = cache_path();
  const size_t slash = path.find_last_of('/');
  if (slash != std::string::npos && slash > 0) mkdir(path.substr(0, slash).c_str(), 0755);
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;  // caching is best effort
  std::fprintf(f, "%s %d %d %u %.3f\n", key.c_str(), mode, block, grid, us);
  std::fclose(f);
}

}  // namespace

// ================================================================== C ABI ==
extern "C" {

int sgp4_version(void) { return 2; }

const char* sgp4_strerror(int code) {
  switch (code) {
    case SGP4_OK: return "ok";
    case SGP4_E_ARG: return "invalid argument (null pointer or inconsistent argument)";
    case SGP4_E_SIZE: return "invalid size (negative or too large n, T or nnz)";
    case SGP4_E_OFFSETS: return "malformed CSR offsets";
    case SGP4_E_PRECISION: return "unknown or unsupported precision";
    case SGP4_E_HIP: return "HIP runtime or launch failure";
    case SGP4_E_GRAVITY: return "gravity model rejected";
    case SGP4_E_PLAN: return "plan does not match the call";
    case SGP4_E_WORKSPACE: return "workspace missing or too small";
    case SGP4_E_HOST: return "host resources exhausted (memory or threads)";
  }
  return "unknown error code";
}

size_t sgp4_consts_bytes(int64_t n) { return n < 0 ? 0 : record_bytes(n); }

int sgp4_init_ex(const double* grav, const double* ref_jd, int64_t n, const double* elem, void* consts,
                 uint8_t* sat_flags, void* stream) {
  if (n < 0 || n > kMaxSats) return SGP4_E_SIZE;
  if (!consts || (n > 0 && !elem)) return SGP4_E_ARG;
  const double* g = grav ? grav : kWgs72;
  if (int rc = check_gravity(g)) return rc;
  double day;
  if (!ref_day_of(ref_jd, &day)) return SGP4_E_ARG;
  return hip_status(launch_init(g, day, n, elem, consts, sat_flags, static_cast<hipStream_t>(stream)));
}

int sgp4_init(const double* grav, int64_t n, const double* elem, void* consts, uint8_t* sat_flags, void* stream) {
  return sgp4_init_ex(grav, nullptr, n, elem, consts, sat_flags, stream);
}

int sgp4_propagate_ex(const void* consts, int64_t n, const double* t, int64_t T, int precision, void* r, void* v,
                      uint8_t* err, int config, void* stream) {
  if (n < 0 || T < 0 || n > kMaxSats || mul_overflows(n, T) || mul_overflows(n * T, 3)) return SGP4_E_SIZE;
  if (precision < 0 || precision > 2) return SGP4_E_PRECISION;
  const int block = config & 0xfff;
  const bool scalar = (config & SGP4_CFG_SCALAR_CONSTS) != 0;
  const bool persistent = (config & SGP4_CFG_PERSISTENT) != 0;
  const bool tiles = (config & SGP4_CFG_TILES) != 0;
  const bool flat = (config & SGP4_CFG_FLAT) != 0;
  const int per_cu = (config >> 20) & 0xff;
  if ((config & ~(0xfff | SGP4_CFG_SCALAR_CONSTS | SGP4_CFG_PERSISTENT | SGP4_CFG_TILES | SGP4_CFG_FLAT |
                  (0xff << 20))) != 0)
    return SGP4_E_ARG;
  if (block != 64 && block != 128 && block != 256 && block != 512) return SGP4_E_ARG;
  if (persistent && per_cu == 0) return SGP4_E_ARG;
  if (tiles && (persistent || !scalar || per_cu != 0)) return SGP4_E_ARG;
  if (flat && (persistent || tiles || scalar || per_cu != 0)) return SGP4_E_ARG;
  if (n == 0 || T == 0) return SGP4_OK;
  if (!consts || !t || !r || !v || !err) return SGP4_E_ARG;
  if (tiles && !dense_tiles_fit(n, T, block)) return SGP4_E_SIZE;
  if (flat && !dense_flat_fits(n, T, block)) return SGP4_E_SIZE;
  if (!tiles && !flat && !persistent && !dense_grid_fits(n, block)) return SGP4_E_SIZE;
  unsigned grid = 0;
  if (persistent) {
    const int64_t tiles = n * ((T + 63) / 64);
    const int64_t need = (tiles + block / 64 - 1) / (block / 64);
    grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(need, int64_t(compute_units()) * per_cu)));
  }
  return hip_status(launch_dense(precision, consts, n, t, T, r, v, err, block, !scalar, grid, tiles, flat,
                                static_cast<hipStream_t>(stream)));
}

int sgp4_propagate(const void* consts, int64_t n, const double* t, int64_t T, int precision, void* r, void* v,
                   uint8_t* err, void* stream) {
  return sgp4_propagate_ex(consts, n, t, T, precision, r, v, err, default_dense(precision, n, T), stream);
}

int sgp4_propagate_elements_ex(const double* grav, const double* ref_jd, int64_t n, const double* elem,
                               const double* t, int64_t T, int precision, void* r, void* v, uint8_t* err,
                               uint8_t* sat_flags, void* ws, size_t ws_bytes, void* stream) {
  if (n < 0 || T < 0 || n > kMaxSats || mul_overflows(n, T) || mul_overflows(n * T, 3)) return SGP4_E_SIZE;
  if (precision < 0 || precision > 2) return SGP4_E_PRECISION;
  const double* g = grav ? grav : kWgs72;
  if (int rc = check_gravity(g)) return rc;
  double day;
  if (!ref_day_of(ref_jd, &day)) return SGP4_E_ARG;
  if (ws && ws_bytes < sgp4_consts_bytes(n)) return SGP4_E_WORKSPACE;
  if (n == 0 || T == 0) return SGP4_OK;
  if (!elem || !t || !r || !v || !err) return SGP4_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (T <= kFusedMaxT || !ws) {
    if (T > fused_max_T()) return SGP4_E_WORKSPACE;
    if (!fused_fits(n, T)) return ws ? SGP4_E_WORKSPACE : SGP4_E_SIZE;
    return hip_status(launch_fused(precision, g, day, n, elem, t, T, r, v, err, sat_flags, s));
  }
  if (int rc = hip_status(launch_init(g, day, n, elem, ws, sat_flags, s))) return rc;
  return sgp4_propagate(ws, n, t, T, precision, r, v, err, stream);
}

int sgp4_propagate_elements(const double* grav, int64_t n, const double* elem, const double* t, int64_t T,
                            int precision, void* r, void* v, uint8_t* err, uint8_t* sat_flags, void* ws,
                            size_t ws_bytes, void* stream) {
  return sgp4_propagate_elements_ex(grav, nullptr, n, elem, t, T, precision, r, v, err, sat_flags, ws, ws_bytes,
                                    stream);
}

size_t sgp4_screen_workspace_bytes(int64_t n, int64_t T) {
  if (n < 0 || T < 0 || mul_overflows(n, T) || mul_overflows(n * T, 16)) return 0;
  return screen_ws_bytes(n, T);
}

int sgp4_screen_ex(const void* r, int precision, const uint8_t* err, int64_t n, int64_t T, double dist_km,
                   int64_t capacity, int32_t* pairs, double* dist, int64_t* count, void* ws, size_t ws_bytes,
                   int mode, void* stream) {
  if (mode < 0 || mode > 2) return SGP4_E_ARG;
  if (n < 0 || T < 0 || T > 0x7ffffff0LL || mul_overflows(n, T) || mul_overflows(n * T, 16) || capacity < 0)
    return SGP4_E_SIZE;
  if ((mode == 1 && n > screen_max_n()) || !screen_global_fits(n, T)) return SGP4_E_SIZE;
  if (precision < 0 || precision > 2) return SGP4_E_PRECISION;
  if (!(dist_km > 0.0) || !std::isfinite(dist_km)) return SGP4_E_ARG;
  if (!count || (capacity > 0 && (!pairs || !dist)) || (n > 0 && T > 0 && !r)) return SGP4_E_ARG;
  if (n >= 2 && T > 0 && (!ws || ws_bytes < screen_ws_bytes(n, T))) return SGP4_E_WORKSPACE;
  return hip_status(launch_screen(r, precision == SGP4_FP64, err, n, T, dist_km, capacity, pairs, dist,
                                  reinterpret_cast<unsigned long long*>(count), ws, mode,
                                  static_cast<hipStream_t>(stream)));
}

int sgp4_screen(const void* r, int precision, const uint8_t* err, int64_t n, int64_t T, double dist_km,
                int64_t capacity, int32_t* pairs, double* dist, int64_t* count, void* ws, size_t ws_bytes,
                void* stream) {
  return sgp4_screen_ex(r, precision, err, n, T, dist_km, capacity, pairs, dist, count, ws, ws_bytes, 0, stream);
}

int sgp4_screen_noalloc(const void* r, int precision, const uint8_t* err, int64_t n, int64_t T, double dist_km,
                        int64_t capacity, int32_t* pairs, double* dist, int64_t* count, void* stream) {
  if (n < 0 || T < 0 || T > 0x7ffffff0LL || mul_overflows(n, T) || mul_overflows(n * T, 16) || capacity < 0)
    return SGP4_E_SIZE;
  if (!screen_global_fits(n, T)) return SGP4_E_SIZE;
  if (n >= 2 && T > 0 && screen_ws_bytes(n, T) > screen_static_bytes()) return SGP4_E_SIZE;
  static_assert(SGP4_SCREEN_NOALLOC_BYTES == 64u << 20, "header limit and scratch size differ");
  if (precision < 0 || precision > 2) return SGP4_E_PRECISION;
  if (!(dist_km > 0.0) || !std::isfinite(dist_km)) return SGP4_E_ARG;
  if (!count || (capacity > 0 && (!pairs || !dist)) || (n > 0 && T > 0 && !r)) return SGP4_E_ARG;
  return hip_status(launch_screen_static(r, precision == SGP4_FP64, err, n, T, dist_km, capacity, pairs, dist,
                                         reinterpret_cast<unsigned long long*>(count),
                                         static_cast<hipStream_t>(stream)));
}

int sgp4_propagate_ragged(const void* consts, int64_t n, const int64_t* offsets, const double* t, int64_t nnz,
                          int precision, void* r, void* v, uint8_t* err, const sgp4_plan* plan, void* stream) {
  if (n < 0 || nnz < 0 || n > kMaxSats || mul_overflows(nnz, 3)) return SGP4_E_SIZE;
  if (precision < 0 || precision > 2) return SGP4_E_PRECISION;
  if (nnz == 0) return SGP4_OK;
  if (n == 0) return SGP4_E_OFFSETS;  // nnz > 0 points cannot belong to no satellite
  if (!consts || !offsets || !t || !r || !v || !err) return SGP4_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan) {
    if (plan->consts != consts || plan->n != n || plan->offsets != offsets || plan->t != t || plan->nnz != nnz ||
        plan->precision != precision || plan->r != r || plan->v != v || plan->err != err)
      return SGP4_E_PLAN;
    return hip_status(plan_launch_direct(plan, s));
  }
  // One wavefront per 64-point chunk (a wavefront that ends after its stores
  // never waits for them); the grid is capped at 2^31 - 1 workgroups, beyond
  // which the wavefronts loop.
  const int64_t nchunks = (nnz + 63) / 64;
  const unsigned grid = unsigned(std::min<int64_t>((nchunks + 3) / 4, int64_t(0xffffffffu / 256)));
  return hip_status(launch_ragged(precision, 1, true, consts, n, offsets, t, nnz, nullptr, nullptr, nchunks, r, v, err, 256,
                                  std::max(grid, 1u), s));
}

static int plan_build(sgp4_plan** out, const void* consts, int64_t n, const int64_t* offsets, const double* t,
                      int64_t nnz, int precision, void* r, void* v, uint8_t* err, unsigned flags, int force_mode,
                      int force_block, int force_per_cu, void* stream) {
  if (!out) return SGP4_E_ARG;
  *out = nullptr;
  if (n <= 0 || nnz <= 0 || n > kMaxSats || mul_overflows(nnz, 3)) return SGP4_E_SIZE;
  if (precision < 0 || precision > 2) return SGP4_E_PRECISION;
  if (!consts || !offsets || !t || !r || !v || !err) return SGP4_E_ARG;
  if (force_mode >= 0 && (force_mode > 1 || (force_block != 64 && force_block != 128 && force_block != 256 &&
                                             force_block != 512) || force_per_cu < 0))
    return SGP4_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<int64_t> off(size_t(n) + 1);
  if (hipMemcpyAsync(off.data(), offsets, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return SGP4_E_HIP;
  if (off[0] != 0 || off[size_t(n)] != nnz) return SGP4_E_OFFSETS;
  for (int64_t i = 0; i < n; ++i)
    if (off[size_t(i) + 1] < off[size_t(i)]) return SGP4_E_OFFSETS;

  // Owned until it is handed out: every early return (and a host allocation
  // failure in the tables below) frees the plan and its device memory.
  struct Owner {
    sgp4_plan* p;
    ~Owner() { plan_free(p); }
  } own{new sgp4_plan};
  sgp4_plan* p = own.p;
  p->precision = precision; p->consts = consts; p->n = n; p->nnz = nnz; p->offsets = offsets; p->t = t;
  p->r = r; p->v = v; p->err = err;

  // Tile tables: tiles of <= 64 points of one satellite; chunk owners for the
  // flat mapping (satellite whose list holds point 64*k).
  std::vector<int64_t> ts;
  std::vector<int32_t> tsat;
  ts.reserve(size_t(nnz / 64 + n));
  tsat.reserve(2 * size_t(nnz / 64 + n));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = off[size_t(i)]; q < off[size_t(i) + 1]; q += 64) {
      ts.push_back(q);
      tsat.push_back(int32_t(i));
      tsat.push_back(int32_t(std::min<int64_t>(64, off[size_t(i) + 1] - q)));
    }
  p->ntiles = int64_t(ts.size());
  p->nchunks = (nnz + 63) / 64;
  std::vector<int32_t> csat(size_t(p->nchunks));
  {
    int64_t i = 0;
    for (int64_t k = 0; k < p->nchunks; ++k) {
      const int64_t q = k * 64;
      while (off[size_t(i) + 1] <= q) ++i;
      csat[size_t(k)] = int32_t(i);
    }
  }
  // Deep-space satellites in the record (one word read back).
  {
    uint32_t* flag = nullptr;
    uint32_t any = 1;
    const bool fok = hipMalloc(&flag, sizeof(uint32_t)) == hipSuccess &&
                     launch_any_deep(consts, n, flag, s) == hipSuccess &&
                     hipMemcpyAsync(&any, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s) == hipSuccess &&
                     hipStreamSynchronize(s) == hipSuccess;
    if (flag) (void)hipFree(flag);
    if (!fok) return SGP4_E_HIP;
    p->deep = any != 0;
  }
  bool ok = hipMalloc(&p->tile_start, ts.size() * sizeof(int64_t)) == hipSuccess &&
            hipMalloc(&p->tile_sat, tsat.size() * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&p->chunk_sat, csat.size() * sizeof(int32_t)) == hipSuccess &&
            hipMemcpyAsync(p->tile_start, ts.data(), ts.size() * sizeof(int64_t), hipMemcpyHostToDevice, s) ==
                hipSuccess &&
            hipMemcpyAsync(p->tile_sat, tsat.data(), tsat.size() * sizeof(int32_t), hipMemcpyHostToDevice, s) ==
                hipSuccess &&
            hipMemcpyAsync(p->chunk_sat, csat.data(), csat.size() * sizeof(int32_t), hipMemcpyHostToDevice, s) ==
                hipSuccess &&
            hipStreamSynchronize(s) == hipSuccess;
  if (!ok) return SGP4_E_HIP;

  const int cus = compute_units();
  auto grid_for = [&](int mode, int block, int per_cu) {
    const int64_t work = mode == 0 ? p->ntiles : p->nchunks;
    const int64_t waves_needed = work;
    const int64_t blocks_needed = (waves_needed + block / 64 - 1) / (block / 64);
    // at most 2^32 - 1 work-items per dispatch; a smaller grid makes the kernels loop
    const int64_t max_grid = std::min<int64_t>(0x7fffffff, int64_t(0xffffffffu) / block);
    return unsigned(std::max<int64_t>(1, std::min({blocks_needed, int64_t(cus) * per_cu, max_grid})));
  };
  // default choice: one wavefront per tile, 256-wide workgroups (fastest on
  // MI355X for the 1M-satellite catalogue in every precision); or the caller's
  // fixed configuration
  p->mode = 0;
  p->block = 256;
  p->grid = grid_for(0, 256, 1 << 30);
  if (force_mode >= 0) {
    p->mode = force_mode;
    p->block = force_block;
    p->grid = grid_for(force_mode, force_block, force_per_cu > 0 ? force_per_cu : (1 << 30));
    flags &= ~unsigned(SGP4_PLAN_AUTOTUNE);
  }

  if (flags & SGP4_PLAN_AUTOTUNE) {
    const std::string key = tune_key(p);
    int m, b;
    unsigned g;
    double us;
    // A cached choice is used only when it is a valid configuration for this
    // batch.
    const bool cached = cache_lookup(key, &m, &b, &g, &us) && m >= 0 && m <= 1 &&
                        (b == 64 || b == 128 || b == 256 || b == 512) && g > 0;
    if (cached) {
      p->mode = m; p->block = b; p->best_us = us;
      p->grid = std::min(g, grid_for(m, b, 1 << 30));
      p->from_cache = true;
    } else {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return SGP4_E_HIP;
      }
      const int blocks[] = {128, 256, 512};
      // waves per CU for the persistent grid; 0 = one wavefront per tile/chunk (no loop)
      const int per_cu[] = {4, 8, 16, 0};
      double best = 1e300;
      for (int mode = 0; mode < 2; ++mode)
        for (int b : blocks)
          for (int pc : per_cu) {
            sgp4_plan c = *p;
            c.mode = mode; c.block = b; c.grid = grid_for(mode, b, pc > 0 ? pc : (1 << 30));
            c.graph = nullptr; c.exec = nullptr;
            if (plan_launch_direct(&c, s) != hipSuccess) continue;  // warm-up
            (void)hipEventRecord(e0, s);
            const int reps = 3;
            bool fine = true;
            for (int k = 0; k < reps; ++k) fine = fine && plan_launch_direct(&c, s) == hipSuccess;
            (void)hipEventRecord(e1, s);
            if (!fine || hipEventSynchronize(e1) != hipSuccess) continue;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double us_c = 1000.0 * ms / reps;
            ++p->ncandidates;
            if (us_c < best) { best = us_c; p->mode = mode; p->block = b; p->grid = c.grid; }
          }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      // nothing of the candidates must stay owned by the copies
      if (p->ncandidates == 0) return SGP4_E_HIP;
      p->best_us = best;
      cache_store(key, p->mode, p->block, p->grid, best);
    }
  }

  if (flags & SGP4_PLAN_GRAPH) {
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return SGP4_E_HIP;
    bool gok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (gok) {
      const hipError_t le = plan_launch_direct(p, cs);
      const hipError_t ce = hipStreamEndCapture(cs, &p->graph);
      gok = le == hipSuccess && ce == hipSuccess &&
            hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
    }
    (void)hipStreamDestroy(cs);
    if (!gok) return SGP4_E_HIP;
  }
  own.p = nullptr;
  *out = p;
  return SGP4_OK;
}

int sgp4_plan_create(sgp4_plan** out, const void* consts, int64_t n, const int64_t* offsets, const double* t,
                     int64_t nnz, int precision, void* r, void* v, uint8_t* err, unsigned flags, void* stream) {
  try {
    return plan_build(out, consts, n, offsets, t, nnz, precision, r, v, err, flags, -1, 0, 0, stream);
  } catch (...) {  // host allocation failure: nothing may unwind through the C ABI
    return SGP4_E_HOST;
  }
}

int sgp4_plan_create_config(sgp4_plan** out, const void* consts, int64_t n, const int64_t* offsets, const double* t,
                            int64_t nnz, int precision, void* r, void* v, uint8_t* err, int mode, int block,
                            int waves_per_cu, unsigned flags, void* stream) {
  if (mode < 0) return SGP4_E_ARG;
  try {
    return plan_build(out, consts, n, offsets, t, nnz, precision, r, v, err, flags, mode, block, waves_per_cu,
                      stream);
  } catch (...) {
    return SGP4_E_HOST;
  }
}

int sgp4_plan_launch(const sgp4_plan* plan, void* stream) {
  if (!plan) return SGP4_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->exec) return hip_status(hipGraphLaunch(plan->exec, s));
  return hip_status(plan_launch_direct(plan, s));
}

int sgp4_plan_describe(const sgp4_plan* plan, char* buf, size_t len) {
  if (!plan || !buf || len == 0) return SGP4_E_ARG;
  std::snprintf(buf, len,
                "{\"mode\": \"%s\", \"block\": %d, \"grid\": %u, \"tiles\": %lld, \"chunks\": %lld, "
                "\"tuned_us\": %.3f, \"candidates\": %d, \"from_cache\": %s, \"graph\": %s, \"near_earth\": %s}",
                plan->mode == 0 ? "tiles" : "flat", plan->block, plan->grid, (long long)plan->ntiles,
                (long long)plan->nchunks, plan->best_us, plan->ncandidates, plan->from_cache ? "true" : "false",
                plan->exec ? "true" : "false", (plan->mode == 0 && !plan->deep) ? "true" : "false");
  return SGP4_OK;
}

void sgp4_plan_destroy(sgp4_plan* plan) { plan_free(plan); }

int sgp4_vjp(int64_t n, const double* elem, const void* consts, const double* t, int64_t T, int precision,
             const void* gr, const void* gv, double* gelem, void* stream) {
  if (n < 0 || T < 0 || n > kMaxSats || mul_overflows(n, T) || mul_overflows(n * T, 3)) return SGP4_E_SIZE;
  if (precision != SGP4_FP64 && precision != SGP4_FP32_MIXED) return SGP4_E_PRECISION;
  if (!grid_fits(uint64_t(n), kVjpLanes)) return SGP4_E_SIZE;  // one workgroup per satellite
  if (n == 0) return SGP4_OK;
  if (!elem || !consts || !gelem || (T > 0 && (!t || !gr))) return SGP4_E_ARG;
  return hip_status(launch_vjp(precision, n, elem, consts, t, T, gr, gv, gelem, static_cast<hipStream_t>(stream)));
}

int sgp4_vjp_ragged(int64_t n, const double* elem, const void* consts, const int64_t* offsets, const double* t,
                    int64_t nnz, int precision, const void* gr, const void* gv, double* gelem, void* stream) {
  if (n < 0 || nnz < 0 || n > kMaxSats || mul_overflows(nnz, 3)) return SGP4_E_SIZE;
  if (precision != SGP4_FP64 && precision != SGP4_FP32_MIXED) return SGP4_E_PRECISION;
  if (!grid_fits(uint64_t(n), kVjpLanes)) return SGP4_E_SIZE;  // one workgroup per satellite
  if (n == 0) return SGP4_OK;
  if (!elem || !consts || !offsets || !gelem || (nnz > 0 && (!t || !gr))) return SGP4_E_ARG;
  return hip_status(launch_vjp_ragged(precision, n, elem, consts, offsets, t, nnz, gr, gv, gelem,
                                      static_cast<hipStream_t>(stream)));
}

int sgp4_jacobian(int64_t n, const double* elem, const void* consts, const double* t, int64_t T, int precision,
                  double* jac, void* stream) {
  if (n < 0 || T < 0 || n > kMaxSats || mul_overflows(n, T) || mul_overflows(n * T, 42)) return SGP4_E_SIZE;
  if (precision != SGP4_FP64 && precision != SGP4_FP32_MIXED) return SGP4_E_PRECISION;
  if (!grid_fits(uint64_t(n), kVjpLanes)) return SGP4_E_SIZE;  // one workgroup per satellite
  if (n == 0 || T == 0) return SGP4_OK;
  if (!elem || !consts || !t || !jac) return SGP4_E_ARG;
  return hip_status(launch_jacobian(precision, n, elem, consts, t, T, jac, static_cast<hipStream_t>(stream)));
}

int sgp4_jacobian_ragged(int64_t n, const double* elem, const void* consts, const int64_t* offsets, const double* t,
                         int64_t nnz, int precision, double* jac, void* stream) {
  if (n < 0 || nnz < 0 || n > kMaxSats || mul_overflows(nnz, 42)) return SGP4_E_SIZE;
  if (precision != SGP4_FP64 && precision != SGP4_FP32_MIXED) return SGP4_E_PRECISION;
  if (!grid_fits(uint64_t(n), kVjpLanes)) return SGP4_E_SIZE;  // one workgroup per satellite
  if (n == 0 || nnz == 0) return SGP4_OK;
  if (!elem || !consts || !offsets || !t || !jac) return SGP4_E_ARG;
  return hip_status(launch_jacobian_ragged(precision, n, elem, consts, offsets, t, nnz, jac,
                                           static_cast<hipStream_t>(stream)));
}

}  // extern "C"

// Conjunction screening on the propagation output: every pair of satellites
// closer than a distance D at a common sample time.
//
// The paper motivates batched propagation by catalogue-wide tasks such as
// conjunction screening (sections 1 and 6) without defining one; this is the
// screening step as defined in the header: at each sample time k, every pair
// i < j of points whose states are valid with
//     d2 = (dx*dx + dy*dy) + dz*dz < D*D,
// dx = x_j - x_i (and so on) formed in double from the stored positions, is an
// event (i, j, k, sqrt(d2)).
//
// Mapping: a packing pass first writes the float x and y of every valid point
// time-major into the workspace (64 x 64 tiles through LDS, so that both the
// reads along times and the writes along satellites are coalesced; invalid
// points get x = +inf).  Then one 1,024-lane workgroup per sample time reads
// its n (x, y) pairs contiguously and counting-sorts the valid points into
// buckets of x of width w >= D plus a rounding margin (at most 4,096 buckets
// over the time's x range; LDS atomics for the counts, one wavefront scan,
// LDS atomics again for the placement).  A partner j of i with
// |x_j - x_i| < D then lies in i's bucket or the next one, so each lane takes
// sorted positions and tests the later points of its bucket and all points
// of the next (on a spherical shell x is uniformly distributed: about
// n 2w / 2R candidates).  A candidate whose float x or y differs by D or more,
// less the rounding margin, is skipped without touching device memory; the
// rest are tested with the full distance from the stored positions.  The
// margin, 1.2e-7 (|a| + |b|) for float roundings a, b of two coordinates,
// bounds the two roundings (2^-24 relative each), so no pair closer than D is
// pruned.  Workgroups are assigned time blocks per XCD (workgroup w runs on
// XCD w mod 8), so the workspace rows of neighbouring times share an L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

namespace sgp4mi {

constexpr int kScreenMaxN = 12288;
constexpr int kScreenBuckets = 4096;
constexpr int kScreenBlock = 1024;

template <class TR>
__device__ __forceinline__ double dist2(const TR* __restrict__ r, int64_t P, int64_t pi, int64_t pj) {
#pragma clang fp contract(off)
  const double dx = double(r[pj]) - double(r[pi]);
  const double dy = double(r[P + pj]) - double(r[P + pi]);
  const double dz = double(r[2 * P + pj]) - double(r[2 * P + pi]);
  return (dx * dx + dy * dy) + dz * dz;
}

// Pack: ws[k * n + i] = (x, y) as floats for a valid point, (+inf, 0) else.
template <class TR>
__global__ void __launch_bounds__(256) screen_pack(const TR* __restrict__ r, const uint8_t* __restrict__ err, int64_t n,
                                                   int64_t T, float2* __restrict__ ws) {
  __shared__ float2 tile[64][65];
  const int64_t k0 = int64_t(blockIdx.x) * 64, i0 = int64_t(blockIdx.y) * 64;  // times on x: T may be large
  const int64_t P = n * T;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int si = e >> 6, kk = e & 63;  // consecutive lanes: consecutive times of one satellite
    const int64_t i = i0 + si, k = k0 + kk;
    float2 v = make_float2(__builtin_inff(), 0.0f);
    if (i < n && k < T) {
      const int64_t p = i * T + k;
      const TR x = r[p], y = r[P + p], z = r[2 * P + p];
      bool ok = isfinite(double(x)) && isfinite(double(y)) && isfinite(double(z));
      if (err) ok = ok && (err[p] == 0 || err[p] == 6);
      if (ok) v = make_float2(float(x), float(y));
    }
    tile[si][kk] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int kk = e >> 6, si = e & 63;  // consecutive lanes: consecutive satellites at one time
    const int64_t i = i0 + si, k = k0 + kk;
    if (i < n && k < T) ws[k * n + i] = tile[si][kk];
  }
}

template <class TR>
__global__ void __launch_bounds__(kScreenBlock)
    screen_kernel(const TR* __restrict__ r, const float2* __restrict__ ws, int32_t n, int64_t T, double D,
                  double D2, int64_t cap, int32_t* __restrict__ pairs, double* __restrict__ dist,
                  unsigned long long* __restrict__ count) {
  // LDS: sorted (x, y)[n], sorted satellite index[n], bucket offsets[kScreenBuckets + 1].
  extern __shared__ float2 smem[];
  float2* oxy = smem;
  uint16_t* oidx = reinterpret_cast<uint16_t*>(oxy + n);
  int32_t* start = reinterpret_cast<int32_t*>(oidx + ((n + 1) & ~1));
  __shared__ float red_lo[kScreenBlock / 64], red_hi[kScreenBlock / 64];
  __shared__ double s_x0, s_inv_w;
  __shared__ int32_t s_nb;
  // XCD-aware time assignment: grid = 8 * per workgroups; workgroup w = 8 q + x
  // (on XCD x) takes time x * per + q, a contiguous block of `per` times per XCD.
  const int64_t per = gridDim.x / 8;
  const int64_t wg = blockIdx.x;
  const int64_t k = (wg % 8) * per + wg / 8;
  if (k >= T) return;  // uniform over the workgroup
  const int64_t P = int64_t(n) * T;
  const float2* wk = ws + k * int64_t(n);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // Range of the valid x.
  float lo = __builtin_inff(), hi = -__builtin_inff();
  for (int32_t s = threadIdx.x; s < n; s += kScreenBlock) {
    const float x = wk[s].x;
    if (x < __builtin_inff()) { lo = fminf(lo, x); hi = fmaxf(hi, x); }
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o));
    hi = fmaxf(hi, __shfl_xor(hi, o));
  }
  if (lane == 0) { red_lo[wave] = lo; red_hi[wave] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < kScreenBlock / 64; ++v) { lo = fminf(lo, red_lo[v]); hi = fmaxf(hi, red_hi[v]); }
    lo = fminf(red_lo[0], lo);
    hi = fmaxf(red_hi[0], hi);
    int32_t nb = 0;
    double x0 = 0.0, inv_w = 0.0;
    if (lo <= hi) {
      const double span = double(hi) - double(lo);
      const double wmin = (D + 2.4e-7 * fmax(fabs(double(lo)), fabs(double(hi)))) * (1.0 + 1.0e-6);
      const double w = fmax(wmin, span / double(kScreenBuckets - 1));
      nb = int32_t(span / w) + 1;
      if (nb > kScreenBuckets) nb = kScreenBuckets;
      x0 = lo;
      inv_w = 1.0 / w;
    }
    s_nb = nb; s_x0 = x0; s_inv_w = inv_w;
  }
  __syncthreads();
  const int32_t nb = s_nb;
  if (nb == 0) return;  // no valid point at this time (uniform)
  const double x0 = s_x0, inv_w = s_inv_w;
  auto bucket = [&](float x) {
    const int32_t b = int32_t((double(x) - x0) * inv_w);
    return b < nb - 1 ? b : nb - 1;
  };

  // Counting sort into buckets: start[b + 1] = count of bucket b, scan, place.
  for (int32_t b = threadIdx.x; b <= nb; b += kScreenBlock) start[b] = 0;
  __syncthreads();
  for (int32_t s = threadIdx.x; s < n; s += kScreenBlock) {
    const float x = wk[s].x;
    if (x < __builtin_inff()) atomicAdd(&start[bucket(x) + 1], 1);
  }
  __syncthreads();
  if (wave == 0) {  // inclusive scan of start[1..nb] by one wavefront
    const int32_t chunk = (nb + 63) / 64;
    const int32_t b0 = 1 + lane * chunk;
    int32_t sum = 0;
    for (int32_t b = b0; b < b0 + chunk && b <= nb; ++b) sum += start[b];
    int32_t incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t u = __shfl_up(incl, o);
      if (lane >= o) incl += u;
    }
    int32_t run = incl - sum;
    for (int32_t b = b0; b < b0 + chunk && b <= nb; ++b) { run += start[b]; start[b] = run; }
  }
  __syncthreads();
  for (int32_t s = threadIdx.x; s < n; s += kScreenBlock) {
    const float2 v = wk[s];
    if (v.x < __builtin_inff()) {
      const int32_t q = atomicAdd(&start[bucket(v.x)], 1);
      oxy[q] = v;
      oidx[q] = uint16_t(s);
    }
  }
  __syncthreads();
  // Now start[b] is the end of bucket b (start[b + 1] before placement).
  const int32_t m = start[nb - 1];

  for (int32_t q = threadIdx.x; q < m; q += kScreenBlock) {
    const float2 vi = oxy[q];
    const int32_t i = oidx[q];
    const int32_t b = bucket(vi.x);
    const int32_t end = b + 1 < nb ? start[b + 1] : start[b];
    const double xi = vi.x, yi = vi.y;
    const int64_t pi = int64_t(i) * T + k;
    for (int32_t q2 = q + 1; q2 < end; ++q2) {
      const float2 vj = oxy[q2];
      const double xj = vj.x, yj = vj.y;
      if (!(fabs(xj - xi) < D + 1.2e-7 * (fabs(xi) + fabs(xj)))) continue;
      if (!(fabs(yj - yi) < D + 1.2e-7 * (fabs(yi) + fabs(yj)))) continue;
      const int32_t j = oidx[q2];
      const int64_t pj = int64_t(j) * T + k;
      const double d2 = dist2(r, P, pi, pj);
      if (d2 < D2) {
        const unsigned long long e = atomicAdd(count, 1ull);
        if (int64_t(e) < cap) {
          pairs[3 * e] = i < j ? i : j;
          pairs[3 * e + 1] = i < j ? j : i;
          pairs[3 * e + 2] = int32_t(k);
          dist[e] = sqrt(d2);
        }
      }
    }
  }
}

__global__ void screen_clear(unsigned long long* count) {
  if (threadIdx.x == 0) *count = 0ull;
}

int screen_max_n() { return kScreenMaxN; }

// Dynamic LDS of the screening kernel: 10 n bytes of sorted points plus the
// bucket offsets (136 KiB at n = 12,288).
static size_t screen_lds_bytes(int64_t n) {
  return size_t(n) * 8 + size_t((n + 1) & ~int64_t(1)) * 2 + size_t(kScreenBuckets + 1) * 4;
}

// ------------------------------------------------------- any-n (global) path --
// The same bucket sort and sweep with the buckets in device memory, for
// batches whose points do not fit one workgroup's LDS.  Buckets of x span a
// range [-R, R] with R the largest |x| of any valid point (one reduction over
// the batch), nb = n / 4 of them at most, width w >= D plus the rounding
// margin of R (fewer, wider buckets when the range is small).  Per time k:
// counts[k][b] (histogram, then offsets by an in-place scan, then ends after
// placement), and the sorted (x, y) and satellite index of the valid points.
struct GHeader {
  unsigned int rbits;  // largest valid |x| as float bits (non-negative floats order as integers)
  int32_t nb;          // buckets in use per time
  double x0, inv_w;    // bucket b = (x - x0) * inv_w
};

struct GLayout {
  GHeader* hdr;
  int32_t* counts;  // [T][nbmax + 1]
  float2* sxy;      // [T][n]
  int32_t* sidx;    // [T][n]
  int64_t nbmax;
};

static int64_t screen_global_buckets(int64_t n) {
  int64_t nb = n / 4;
  if (nb < 16) nb = 16;
  if (nb > (int64_t(1) << 20)) nb = int64_t(1) << 20;
  return nb;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static GLayout global_layout(void* ws, int64_t n, int64_t T) {
  GLayout L;
  L.nbmax = screen_global_buckets(n);
  char* b = static_cast<char*>(ws);
  L.hdr = reinterpret_cast<GHeader*>(b);
  b += align256(sizeof(GHeader));
  L.counts = reinterpret_cast<int32_t*>(b);
  b += align256(size_t(T) * size_t(L.nbmax + 1) * 4);
  L.sxy = reinterpret_cast<float2*>(b);
  b += align256(size_t(T) * size_t(n) * 8);
  L.sidx = reinterpret_cast<int32_t*>(b);
  return L;
}

static size_t global_ws_bytes(int64_t n, int64_t T) {
  const int64_t nbmax = screen_global_buckets(n);
  return align256(sizeof(GHeader)) + align256(size_t(T) * size_t(nbmax + 1) * 4) + align256(size_t(T) * size_t(n) * 8) +
         size_t(T) * size_t(n) * 4;
}

template <class TR>
__device__ __forceinline__ bool valid_point(const TR* __restrict__ r, const uint8_t* __restrict__ err, int64_t P,
                                            int64_t p, float* x, float* y) {
  const TR vx = r[p], vy = r[P + p], vz = r[2 * P + p];
  bool ok = isfinite(double(vx)) && isfinite(double(vy)) && isfinite(double(vz));
  if (err) ok = ok && (err[p] == 0 || err[p] == 6);
  *x = float(vx);
  *y = float(vy);
  return ok;
}

// Clear the header and the counts (a fill kernel, so the launch sequence can
// be captured in a graph).
__global__ void gscreen_clear(GLayout L, int64_t T) {
  const int64_t total = T * (L.nbmax + 1);
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < total; q += int64_t(gridDim.x) * blockDim.x)
    L.counts[q] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    L.hdr->rbits = 0u;
    L.hdr->nb = 0;
  }
}

template <class TR>
__global__ void __launch_bounds__(256) gscreen_range(const TR* __restrict__ r, const uint8_t* __restrict__ err,
                                                     int64_t P, GLayout L) {
  float m = 0.0f;
  for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < P; p += int64_t(gridDim.x) * 256) {
    float x, y;
    if (valid_point(r, err, P, p, &x, &y)) m = fmaxf(m, fabsf(x));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(&L.hdr->rbits, __float_as_uint(m));
}

__global__ void gscreen_buckets(GLayout L, double D) {
  if (threadIdx.x != 0) return;
  const double R = double(__uint_as_float(L.hdr->rbits));
  const double span = 2.0 * R;
  const double w = fmax((D + 2.4e-7 * R) * (1.0 + 1.0e-6), span / double(L.nbmax - 1));
  int64_t nb = int64_t(span / w) + 1;
  if (nb > L.nbmax) nb = L.nbmax;
  L.hdr->nb = int32_t(nb);
  L.hdr->x0 = -R;
  L.hdr->inv_w = 1.0 / w;
}

__device__ __forceinline__ int32_t gbucket(const GHeader& h, float x) {
  const int32_t b = int32_t((double(x) - h.x0) * h.inv_w);
  return b < h.nb - 1 ? b : h.nb - 1;
}

template <class TR>
__global__ void __launch_bounds__(256) gscreen_count(const TR* __restrict__ r, const uint8_t* __restrict__ err,
                                                     int64_t T, int64_t P, GLayout L) {
  const GHeader h = *L.hdr;
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= P) return;
  float x, y;
  if (!valid_point(r, err, P, p, &x, &y)) return;
  const int64_t k = p % T;
  atomicAdd(&L.counts[k * (L.nbmax + 1) + gbucket(h, x) + 1], 1);
}

// Inclusive scan of counts[k][1..nb] per time (one workgroup per time, 256
// lanes, chunks of 256 buckets with a running carry).
__global__ void __launch_bounds__(256) gscreen_scan(GLayout L) {
  __shared__ int32_t part[4];
  __shared__ int32_t carry_s;
  const int32_t nb = L.hdr->nb;
  int32_t* c = L.counts + int64_t(blockIdx.x) * (L.nbmax + 1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t carry = 0;
  for (int32_t base = 1; base <= nb; base += 256) {
    const int32_t b = base + int32_t(threadIdx.x);
    int32_t v = b <= nb ? c[b] : 0;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    if (lane == 63) part[wave] = v;
    __syncthreads();
    int32_t before = carry;
    for (int q = 0; q < wave; ++q) before += part[q];
    if (b <= nb) c[b] = before + v;
    if (threadIdx.x == 255) carry_s = before + v;
    __syncthreads();
    carry = carry_s;
    __syncthreads();
  }
}

template <class TR>
__global__ void __launch_bounds__(256) gscreen_place(const TR* __restrict__ r, const uint8_t* __restrict__ err,
                                                     int64_t n, int64_t T, GLayout L) {
  const GHeader h = *L.hdr;
  const int64_t P = n * T;
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= P) return;
  float x, y;
  if (!valid_point(r, err, P, p, &x, &y)) return;
  const int64_t i = p / T, k = p - (p / T) * T;
  const int32_t q = atomicAdd(&L.counts[k * (L.nbmax + 1) + gbucket(h, x)], 1);
  L.sxy[k * n + q] = make_float2(x, y);
  L.sidx[k * n + q] = int32_t(i);
}

template <class TR>
__global__ void __launch_bounds__(256)
    gscreen_sweep(const TR* __restrict__ r, int64_t n, int64_t T, double D, double D2, GLayout L, int64_t cap,
                  int32_t* __restrict__ pairs, double* __restrict__ dist, unsigned long long* __restrict__ count) {
  const GHeader h = *L.hdr;
  const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (g >= n * T) return;
  const int64_t k = g / n, q = g - (g / n) * n;
  const int32_t* c = L.counts + k * (L.nbmax + 1);
  if (q >= c[h.nb - 1]) return;  // after placement c[b] is the end of bucket b
  const float2* sxy = L.sxy + k * n;
  const int32_t* sidx = L.sidx + k * n;
  const int64_t P = n * T;
  const float2 vi = sxy[q];
  const int32_t i = sidx[q];
  const int32_t b = gbucket(h, vi.x);
  const int32_t end = b + 1 < h.nb ? c[b + 1] : c[b];
  const double xi = vi.x, yi = vi.y;
  const int64_t pi = int64_t(i) * T + k;
  // candidates in groups of eight: the group's loads are issued together (a
  // position past the bucket's end reads as NaN and fails the tests)
  constexpr int kU = 8;
  for (int32_t q0 = int32_t(q) + 1; q0 < end; q0 += kU) {
    float2 vj[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      vj[u] = q0 + u < end ? sxy[q0 + u] : make_float2(__builtin_nanf(""), __builtin_nanf(""));
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const double xj = vj[u].x, yj = vj[u].y;
      if (!(fabs(xj - xi) < D + 1.2e-7 * (fabs(xi) + fabs(xj)))) continue;
      if (!(fabs(yj - yi) < D + 1.2e-7 * (fabs(yi) + fabs(yj)))) continue;
      const int32_t j = sidx[q0 + u];
      const int64_t pj = int64_t(j) * T + k;
      const double d2 = dist2(r, P, pi, pj);
      if (d2 < D2) {
        const unsigned long long e = atomicAdd(count, 1ull);
        if (int64_t(e) < cap) {
          pairs[3 * e] = i < j ? i : j;
          pairs[3 * e + 1] = i < j ? j : i;
          pairs[3 * e + 2] = int32_t(k);
          dist[e] = sqrt(d2);
        }
      }
    }
  }
}

template <class TR>
static hipError_t screen_global(const TR* r, const uint8_t* err, int64_t n, int64_t T, double D, int64_t cap,
                                int32_t* pairs, double* dist, unsigned long long* count, void* ws, hipStream_t s) {
  const GLayout L = global_layout(ws, n, T);
  const int64_t P = n * T;
  const unsigned gp = unsigned((P + 255) / 256);
  const int64_t cells = T * (L.nbmax + 1);
  hipLaunchKernelGGL(gscreen_clear, dim3(unsigned(std::min<int64_t>((cells + 255) / 256, 65536))), dim3(256), 0, s,
                     L, T);
  hipLaunchKernelGGL(gscreen_range<TR>, dim3(unsigned(std::min<int64_t>((P + 255) / 256, 16384))), dim3(256), 0, s,
                     r, err, P, L);
  hipLaunchKernelGGL(gscreen_buckets, dim3(1), dim3(64), 0, s, L, D);
  hipLaunchKernelGGL(gscreen_count<TR>, dim3(gp), dim3(256), 0, s, r, err, T, P, L);
  hipLaunchKernelGGL(gscreen_scan, dim3(unsigned(T)), dim3(256), 0, s, L);
  hipLaunchKernelGGL(gscreen_place<TR>, dim3(gp), dim3(256), 0, s, r, err, n, T, L);
  hipLaunchKernelGGL(gscreen_sweep<TR>, dim3(gp), dim3(256), 0, s, r, n, T, D, D * D, L, cap, pairs, dist, count);
  return hipGetLastError();
}

// Workspace of the two paths: the LDS path packs 8 bytes per point; the
// global path holds the header, the per-time bucket offsets and 12 bytes per
// point of sorted (x, y) and satellite index.
size_t screen_ws_bytes(int64_t n, int64_t T) {
  const size_t lds = size_t(n) * size_t(T) * sizeof(float2);
  const size_t glob = global_ws_bytes(n, T);
  return lds > glob ? lds : glob;  // enough for either path
}

// Largest n * T the global path indexes (grids of 256-lane workgroups).
bool screen_global_fits(int64_t n, int64_t T) {
  return n <= 0x7fffffff && n * T <= int64_t(0x7fffffff) * 256 && T <= 0x7fffffff;
}

// mode 0: the LDS path when n <= kScreenMaxN, else the global path; 1: LDS
// path (the caller checks n); 2: global path.
hipError_t launch_screen(const void* r, bool fp64, const uint8_t* err, int64_t n, int64_t T, double D, int64_t cap,
                         int32_t* pairs, double* dist, unsigned long long* count, void* ws, int mode, hipStream_t s) {
  hipLaunchKernelGGL(screen_clear, dim3(1), dim3(64), 0, s, count);
  if (n < 2 || T == 0) return hipGetLastError();
  if (mode == 2 || (mode == 0 && n > kScreenMaxN)) {
    if (fp64) return screen_global(static_cast<const double*>(r), err, n, T, D, cap, pairs, dist, count, ws, s);
    return screen_global(static_cast<const float*>(r), err, n, T, D, cap, pairs, dist, count, ws, s);
  }
  float2* w = static_cast<float2*>(ws);
  const dim3 pg(unsigned((T + 63) / 64), unsigned((n + 63) / 64));
  if (fp64)
    hipLaunchKernelGGL(screen_pack<double>, pg, dim3(256), 0, s, static_cast<const double*>(r), err, n, T, w);
  else
    hipLaunchKernelGGL(screen_pack<float>, pg, dim3(256), 0, s, static_cast<const float*>(r), err, n, T, w);
  const unsigned grid = unsigned(8 * ((T + 7) / 8));
  const size_t lds = screen_lds_bytes(n);
  static bool attr_set = false;
  if (!attr_set) {
    const int most = int(screen_lds_bytes(kScreenMaxN));
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&screen_kernel<double>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, most);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&screen_kernel<float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, most);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (fp64)
    hipLaunchKernelGGL(screen_kernel<double>, dim3(grid), dim3(kScreenBlock), lds, s, static_cast<const double*>(r),
                       w, int32_t(n), T, D, D * D, cap, pairs, dist, count);
  else
    hipLaunchKernelGGL(screen_kernel<float>, dim3(grid), dim3(kScreenBlock), lds, s, static_cast<const float*>(r), w,
                       int32_t(n), T, D, D * D, cap, pairs, dist, count);
  return hipGetLastError();
}

// ------------------------------------------------------------- no-alloc --
// Workspace for callers that cannot allocate device memory: a fixed array in
// the code object, one copy per GPU the library runs on, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host it names a stand-in, not device memory); it passes the device address
// taken with hipGetSymbolAddress once per device, with that device current.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

size_t screen_static_bytes() { return kStaticScratchBytes; }

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// This GPU's copy of the scratch array (the current device's), looked up on
// the first call on that device.
static hipError_t scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// launch_screen (mode 0) with the workspace in this GPU's scratch array; the
// caller checks that screen_ws_bytes(n, T) fits kStaticScratchBytes.  Both
// paths initialise every workspace byte they read (the packing pass writes
// all n T entries; the device-memory path clears its header and counts with a
// kernel), so nothing of an earlier call's contents is used.
hipError_t launch_screen_static(const void* r, bool fp64, const uint8_t* err, int64_t n, int64_t T, double D,
                                int64_t cap, int32_t* pairs, double* dist, unsigned long long* count, hipStream_t s) {
  void* ws = nullptr;
  if (hipError_t e = scratch_of_current_device(&ws)) return e;
  return launch_screen(r, fp64, err, n, T, D, cap, pairs, dist, count, ws, 0, s);
}

}  // namespace sgp4mi

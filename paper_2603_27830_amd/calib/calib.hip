// Calibration microbenchmarks for the roofline: the issue rate of plain
// (unpacked) FP64 and FP32 fused multiply-adds, and the bandwidth of a
// non-temporal store stream.  Measurement support only; the propagation
// library does not use this file.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

template <class T>
__global__ void __launch_bounds__(256) fma_loop(T* out, int iters, T a, T b) {
  T acc[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) acc[k] = T(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc[k] = acc[k] * a + b;
  }
  T s = T(0);
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += acc[k];
  out[size_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

template <class T>
__global__ void __launch_bounds__(256) store_nt(T* buf, size_t n, T x) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(x + T(i & 7), buf + i);
}

}  // namespace

extern "C" {

// out: device array of blocks*256 elements.  flop = blocks*256*iters*8*2.
int sgp4mi_calib_fma(int precision, void* out, int blocks, int iters, void* stream) {
  if (!out || blocks <= 0 || iters <= 0) return -1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == 0)
    hipLaunchKernelGGL(fma_loop<double>, dim3(blocks), dim3(256), 0, s, static_cast<double*>(out), iters,
                       0.999999999, 1e-9);
  else
    hipLaunchKernelGGL(fma_loop<float>, dim3(blocks), dim3(256), 0, s, static_cast<float*>(out), iters, 0.9999f,
                       1e-4f);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

// buf: device array of n doubles, written once with non-temporal stores.
int sgp4mi_calib_store(void* buf, size_t n, int blocks, void* stream) {
  if (!buf || blocks <= 0) return -1;
  hipLaunchKernelGGL(store_nt<double>, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<double*>(buf), n, 1.0);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"

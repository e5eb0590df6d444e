// Calibration microbenchmarks for the roofline: the issue rate of plain
// (unpacked) FP64 and FP32 fused multiply-adds, and the bandwidth of a
// non-temporal store stream.  FP32 is measured twice: all operands in vector
// registers, and with one operand in a scalar register (on gfx950 the second
// issues at about half the rate of the first).  Measurement support only; the
// propagation library does not use this file.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

// kVgpr: copy the multiplier into a vector register first (the empty asm
// keeps the compiler from folding it back into the scalar kernel argument).
template <class T, bool kVgpr>
__global__ void __launch_bounds__(256) fma_loop(T* out, int iters, T a, T b) {
  T acc[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) acc[k] = T(threadIdx.x + k);
  if (kVgpr) asm volatile("" : "+v"(a));
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc[k] = acc[k] * a + b;
  }
  T s = T(0);
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += acc[k];
  out[size_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

// Issue rate of single instructions: 8 independent chains per lane of one
// instruction kind, written as inline assembly so the kind and its operand
// registers are exactly the ones named.
constexpr int kRateKinds = 8;
template <int kKind>
__global__ void __launch_bounds__(256) rate_loop(float* out, int iters, float a) {
  float x[kChains];
  double y[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    x[k] = float(threadIdx.x + k + 1) * 1e-3f;
    y[k] = double(x[k]);
  }
  float va = a;
  asm volatile("" : "+v"(va));
  const float sa = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, a)));
  const double vd = double(va);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
      if constexpr (kKind == 0) asm volatile("v_fma_f32 %0, %0, %1, %0" : "+v"(x[k]) : "v"(va));
      if constexpr (kKind == 1) asm volatile("v_fma_f32 %0, %1, %0, %2" : "+v"(x[k]) : "s"(sa), "v"(va));
      if constexpr (kKind == 2) asm volatile("v_mul_f32 %0, %1, %0" : "+v"(x[k]) : "v"(va));
      if constexpr (kKind == 3) asm volatile("v_fma_f64 %0, %0, %1, %0" : "+v"(y[k]) : "v"(vd));
      if constexpr (kKind == 4) asm volatile("v_sin_f32 %0, %0" : "+v"(x[k]));
      if constexpr (kKind == 5) asm volatile("v_rcp_f32 %0, %0" : "+v"(x[k]));
      if constexpr (kKind == 6) asm volatile("v_rcp_f64 %0, %0" : "+v"(y[k]));
      if constexpr (kKind == 7) asm volatile("v_cvt_f32_f64 %0, %1" : "=v"(x[k]) : "v"(y[k]));
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += x[k] + float(y[k]);
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

// out: device array of blocks*256 elements (double for precision 0, float
// otherwise).  precision 0: FP64; 1: FP32, vector-register operands; 2: FP32,
// multiplier in a scalar register.  flop = blocks*256*iters*8*2.
int sgp4mi_calib_fma(int precision, void* out, int blocks, int iters, void* stream) {
  if (!out || blocks <= 0 || iters <= 0 || precision < 0 || precision > 2) return -1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == 0)
    hipLaunchKernelGGL((fma_loop<double, true>), dim3(blocks), dim3(256), 0, s, static_cast<double*>(out), iters,
                       0.999999999, 1e-9);
  else if (precision == 1)
    hipLaunchKernelGGL((fma_loop<float, true>), dim3(blocks), dim3(256), 0, s, static_cast<float*>(out), iters,
                       0.9999f, 1e-4f);
  else
    hipLaunchKernelGGL((fma_loop<float, false>), dim3(blocks), dim3(256), 0, s, static_cast<float*>(out), iters,
                       0.9999f, 1e-4f);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

// out: device float array of blocks*256 elements.  kind: 0 v_fma_f32 (vector
// operands), 1 v_fma_f32 (one scalar operand), 2 v_mul_f32, 3 v_fma_f64,
// 4 v_sin_f32, 5 v_rcp_f32, 6 v_rcp_f64, 7 v_cvt_f32_f64.  Instructions issued
// = blocks * 4 wavefronts * iters * 8.
int sgp4mi_calib_rate(int kind, void* out, int blocks, int iters, void* stream) {
  if (!out || blocks <= 0 || iters <= 0 || kind < 0 || kind >= kRateKinds) return -1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* o = static_cast<float*>(out);
  switch (kind) {
    case 0: hipLaunchKernelGGL(rate_loop<0>, dim3(blocks), dim3(256), 0, s, o, iters, 0.999f); break;
    case 1: hipLaunchKernelGGL(rate_loop<1>, dim3(blocks), dim3(256), 0, s, o, iters, 0.999f); break;
    case 2: hipLaunchKernelGGL(rate_loop<2>, dim3(blocks), dim3(256), 0, s, o, iters, 0.999f); break;
    case 3: hipLaunchKernelGGL(rate_loop<3>, dim3(blocks), dim3(256), 0, s, o, iters, 0.999f); break;
    case 4: hipLaunchKernelGGL(rate_loop<4>, dim3(blocks), dim3(256), 0, s, o, iters, 0.999f); break;
    case 5: hipLaunchKernelGGL(rate_loop<5>, dim3(blocks), dim3(256), 0, s, o, iters, 0.999f); break;
    case 6: hipLaunchKernelGGL(rate_loop<6>, dim3(blocks), dim3(256), 0, s, o, iters, 0.999f); break;
    default: hipLaunchKernelGGL(rate_loop<7>, dim3(blocks), dim3(256), 0, s, o, iters, 0.999f); break;
  }
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

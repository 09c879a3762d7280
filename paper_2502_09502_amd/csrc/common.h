// Shared device/host helpers for the certglm HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdio>
#include <string>

namespace cgl {

constexpr int kWave = 64;

// ---------------------------------------------------------------- error plumbing (host)

void set_error(const std::string& msg);  // thread-local detail string (api.cpp)

struct HipError {
  hipError_t err;
  const char* what;
};

#define CGL_HIP(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) throw ::cgl::HipError{e_, #expr};                  \
  } while (0)

// ---------------------------------------------------------------- wave / block reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ uint64_t wave_and(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v &= __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide reductions. `scratch` must hold blockDim/64 entries of the value type; all threads
// of the block must call. The result is returned to every thread.
template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, T* scratch, Op op, T init) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off, kWave));
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  T r = init;
  for (int i = 0; i < nw; ++i) r = op(r, scratch[i]);
  return r;
}

struct OpAdd {
  template <typename T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
  template <typename T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a > b ? a : b; }
};
struct OpMin {
  template <typename T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a < b ? a : b; }
};
struct OpOr {
  __device__ __forceinline__ uint64_t operator()(uint64_t a, uint64_t b) const { return a | b; }
};
struct OpAnd {
  __device__ __forceinline__ uint64_t operator()(uint64_t a, uint64_t b) const { return a & b; }
};

// ---------------------------------------------------------------- element conversions

__device__ __forceinline__ double bf16_to_double(uint16_t b) {
  return (double)__uint_as_float(((uint32_t)b) << 16);
}
__device__ __forceinline__ float bf16_to_float(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}
// Round-to-nearest-even float -> bfloat16 bits (finite inputs).
__device__ __forceinline__ uint16_t float_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename T>
struct XLoad;
template <>
struct XLoad<double> {
  static __device__ __forceinline__ double get(const double* p, size_t i) { return p[i]; }
};
template <>
struct XLoad<float> {
  static __device__ __forceinline__ double get(const float* p, size_t i) { return (double)p[i]; }
};
template <>
struct XLoad<uint16_t> {
  static __device__ __forceinline__ double get(const uint16_t* p, size_t i) {
    return bf16_to_double(p[i]);
  }
};

// ---------------------------------------------------------------- scalar maths of the method

// Huber H_M (Sec. 3.1) of |a|.
__device__ __host__ __forceinline__ double huber(double a, double M) {
  a = fabs(a);
  return a <= M ? 0.5 * a * a : M * a - 0.5 * M * M;
}
// argmin_nu 1/2 (nu - x)^2 + c H_M(nu) for x >= 0 (block value of Alg. 1).
__device__ __host__ __forceinline__ double huber_prox(double c, double x, double M) {
  return x <= M * (1.0 + c) ? x / (1.0 + c) : x - c * M;
}

}  // namespace cgl

// Shared device/host helpers for the certglm HIP library (gfx950, wave64).
#pragma once

#include <climits>

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
//
// Reductions over the 64 lanes of a wave use DPP row operations (register-to-register, no LDS
// round trip): pairs and quads by quad permutations, rows of 16 by row shifts of 4 and 8, then
// rows 1 and 3 take the last lane of the row below (row broadcast 15) and rows 2 and 3 take
// lane 31 (row broadcast 31), which leaves the total in lane 63; it is then read back as a
// wave-uniform value. Lanes whose DPP source is outside the pattern receive the identity. The
// combination order is fixed, so results are deterministic. Every lane of the wave must be
// active.

template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_move(T ident, T v) {
  static_assert(sizeof(T) % 4 == 0, "32-bit words");
  constexpr int W = sizeof(T) / 4;
  int a[W], b[W];
  __builtin_memcpy(a, &ident, sizeof(T));
  __builtin_memcpy(b, &v, sizeof(T));
#pragma unroll
  for (int w = 0; w < W; ++w) a[w] = __builtin_amdgcn_update_dpp(a[w], b[w], CTRL, ROWS, 0xF, false);
  T r;
  __builtin_memcpy(&r, a, sizeof(T));
  return r;
}

template <typename T>
__device__ __forceinline__ T read_lane63(T v) {
  constexpr int W = sizeof(T) / 4;
  int a[W];
  __builtin_memcpy(a, &v, sizeof(T));
#pragma unroll
  for (int w = 0; w < W; ++w) a[w] = __builtin_amdgcn_readlane(a[w], 63);
  T r;
  __builtin_memcpy(&r, a, sizeof(T));
  return r;
}

template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, T ident, Op op) {
  v = op(v, dpp_move<0xB1, 0xF>(ident, v));   // quad_perm [1, 0, 3, 2]
  v = op(v, dpp_move<0x4E, 0xF>(ident, v));   // quad_perm [2, 3, 0, 1]
  v = op(v, dpp_move<0x114, 0xF>(ident, v));  // row_shr 4
  v = op(v, dpp_move<0x118, 0xF>(ident, v));  // row_shr 8
  v = op(v, dpp_move<0x142, 0xA>(ident, v));  // row_bcast 15 into rows 1 and 3
  v = op(v, dpp_move<0x143, 0xC>(ident, v));  // row_bcast 31 into rows 2 and 3
  return read_lane63(v);
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

__device__ __forceinline__ double wave_sum(double v) { return wave_reduce(v, 0.0, OpAdd()); }
__device__ __forceinline__ float wave_sum(float v) { return wave_reduce(v, 0.0f, OpAdd()); }
__device__ __forceinline__ int wave_sum(int v) { return wave_reduce(v, 0, OpAdd()); }
__device__ __forceinline__ int wave_max(int v) { return wave_reduce(v, INT_MIN, OpMax()); }
__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, -HUGE_VAL, OpMax());
}
__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
  return wave_reduce(v, (uint64_t)0, OpOr());
}
__device__ __forceinline__ uint64_t wave_and(uint64_t v) {
  return wave_reduce(v, ~(uint64_t)0, OpAnd());
}

// Block-wide reductions. `scratch` must hold blockDim/64 entries of the value type; all threads
// of the block must call; init is the identity of op. The result is returned to every thread.
template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, T* scratch, Op op, T init) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  v = wave_reduce(v, init, op);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  T r = init;
  for (int i = 0; i < nw; ++i) r = op(r, scratch[i]);
  return r;
}

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

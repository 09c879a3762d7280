// FP64 MFMA product of the certification rounds: C[q][m] = sum_{k < K} A[m][k] * B[q][k].
//
//   A: M x K row-major in the design's stored precision (BF16 bits, FP32 or FP64), lda >= K
//      rounded up to 16; every element is widened to FP64 exactly before the product;
//   B: Q x K FP64 row-major (one row per certified node), ldb >= K rounded up to 16;
//   C: FP64, node-major (ldc). With split-K the chunks write Q x M partials that a second
//      kernel sums in a fixed order, so the result does not depend on scheduling.
//
// One wave computes a (16 F64_RT)-row x 16*NT-node block with v_mfma_f64_16x16x4f64 and needs
// no LDS and no barrier. The k index of each MFMA is permuted so that every lane's operands are
// contiguous in memory: in the 16-wide k-step at k0, lane (i, kk) (i = lane % 16,
// kk = lane / 16) holds k0 + 4 kk + s for MFMA sub-step s, for A (row i) and B (node i) alike,
// which leaves the contraction unchanged. A and B fragments go straight from global memory
// into registers, F64_PD steps ahead. Elements past the end of the k-range (padding, whose
// contents are not guaranteed, and the re-read steps that pad the loop) are replaced by zero
// before they enter a product.
#pragma once

#include "common.h"

namespace cgl {

constexpr int F64_PD = 2;  // 16-wide k-steps in flight per wave
constexpr int F64_RT = 4;  // row tiles of 16 per wave

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64acc4;

// Four consecutive A elements along k, loaded with one vector load and widened one by one.
template <typename XT>
struct F64Frag;
template <>
struct F64Frag<uint16_t> {
  typedef unsigned int raw __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ raw load(const uint16_t* p) {
    return *reinterpret_cast<const raw*>(p);
  }
  static __device__ __forceinline__ double get(const raw& v, int e) {
    const unsigned w = v[e >> 1];
    return (double)__uint_as_float((e & 1) ? (w & 0xffff0000u) : (w << 16));
  }
};
template <>
struct F64Frag<float> {
  typedef float raw __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ raw load(const float* p) {
    return *reinterpret_cast<const raw*>(p);
  }
  static __device__ __forceinline__ double get(const raw& v, int e) { return (double)v[e]; }
};
template <>
struct F64Frag<double> {
  typedef double raw __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ raw load(const double* p) {
    return *reinterpret_cast<const raw*>(p);
  }
  static __device__ __forceinline__ double get(const raw& v, int e) { return v[e]; }
};

struct F64GemmArgs {
  const void* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  int64_t M, K;
  int Q;
  int64_t kchunk;  // split-K chunk, a multiple of 16
  double* C;       // final result (ksplit == 1) or Q x M partials per chunk (ksplit > 1)
  int64_t ldc;
};

template <typename XT, int NT>
__global__ __launch_bounds__(256) void k_gemm_f64(F64GemmArgs g) {
  typedef F64Frag<XT> FA;
  typedef typename F64Frag<double>::raw b4;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t m0 = ((int64_t)blockIdx.x * 4 + wid) * (16 * F64_RT);
  if (m0 >= g.M) return;  // no barrier below: a wave past the last row may leave at once
  const int q0 = (int)blockIdx.y * 16 * NT;
  const int64_t kb = (int64_t)blockIdx.z * g.kchunk;
  const int64_t ke = min(kb + g.kchunk, g.K);
  const int li = lane & 15;
  const int kk = lane >> 4;
  // rows and nodes past the end are clamped to the last valid one (their results are dropped)
  const XT* ap[F64_RT];
#pragma unroll
  for (int r = 0; r < F64_RT; ++r)
    ap[r] = (const XT*)g.A + min(m0 + 16 * r + li, g.M - 1) * g.lda + kb + 4 * kk;
  const double* bp[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
    bp[t] = g.B + (int64_t)min(q0 + 16 * t + li, g.Q - 1) * g.ldb + kb + 4 * kk;

  f64acc4 acc[F64_RT][NT];
#pragma unroll
  for (int r = 0; r < F64_RT; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[r][t][e] = 0.0;

  const int nsteps = (int)((ke - kb + 15) / 16);
  if (nsteps > 0) {
    // the step count is padded to a multiple of F64_PD so the unrolled body has no branches;
    // padded steps re-read the last step (a valid address) and are masked to zero
    const int nsp = (nsteps + F64_PD - 1) / F64_PD * F64_PD;
    const int64_t last = (int64_t)(nsteps - 1) * 16;
    typename FA::raw ra[F64_PD][F64_RT];
    b4 rb[F64_PD][NT];
#pragma unroll
    for (int d = 0; d < F64_PD; ++d) {
      const int64_t o = min((int64_t)d * 16, last);
#pragma unroll
      for (int r = 0; r < F64_RT; ++r) ra[d][r] = FA::load(ap[r] + o);
#pragma unroll
      for (int t = 0; t < NT; ++t) rb[d][t] = *reinterpret_cast<const b4*>(bp[t] + o);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int s = 0; s < nsp; s += F64_PD) {
#pragma unroll
      for (int d = 0; d < F64_PD; ++d) {
        __builtin_amdgcn_sched_barrier(0);
        const int64_t kl = kb + (int64_t)(s + d) * 16 + 4 * kk;  // this lane's first k
        double a[F64_RT][4], b[NT][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = kl + e < ke;
#pragma unroll
          for (int r = 0; r < F64_RT; ++r) a[r][e] = ok ? FA::get(ra[d][r], e) : 0.0;
#pragma unroll
          for (int t = 0; t < NT; ++t) b[t][e] = ok ? rb[d][t][e] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int r = 0; r < F64_RT; ++r)
#pragma unroll
            for (int t = 0; t < NT; ++t)
              acc[r][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r][e], b[t][e], acc[r][t], 0, 0, 0);
        const int64_t o = min((int64_t)(s + d + F64_PD) * 16, last);
#pragma unroll
        for (int r = 0; r < F64_RT; ++r) ra[d][r] = FA::load(ap[r] + o);
#pragma unroll
        for (int t = 0; t < NT; ++t) rb[d][t] = *reinterpret_cast<const b4*>(bp[t] + o);
      }
    }
  }
  // C tile element (i, j) sits in lane j + 16 (i % 4), accumulator element i / 4
  double* C = g.C + (int64_t)blockIdx.z * g.Q * g.ldc;
#pragma unroll
  for (int r = 0; r < F64_RT; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t m = m0 + 16 * r + kk + 4 * e;
        const int q = q0 + 16 * t + li;
        if (m < g.M && q < g.Q) C[(int64_t)q * g.ldc + m] = acc[r][t][e];
      }
}

// Row-gathered form for a right-hand side with few nonzero coordinates:
//   C[q][m] = sum_{u < K} At[idx[u]][m] * B[q][u],
//   At: the transposed design (one row per coordinate, row-major, ldat a multiple of 256 that
//       covers every row m of the product), in the stored precision;
//   idx: the K coordinates kept, readable up to K rounded up to 16 (entries past K name a valid
//        row; their terms are replaced by zero); K may be read from device memory at launch;
//   B: Q x K FP64, the right-hand sides compacted to those coordinates (ldb >= K rounded up to 16).
// When every coordinate left out is zero in every right-hand side, this is the full product of
// the design with the uncompacted right-hand sides, up to the order of the FP64 sum.
//
// Lane (i, kk) holds rows m0 + 4 i + r of the wave's 64 rows for row tile r, so one vector load
// of four consecutive elements of a row of At feeds all four row tiles; the k index of sub-step
// s is k0 + 4 kk + s, as in k_gemm_f64. The row indices of a step are loaded F64_PD steps before
// its A fragments.
struct F64RowsArgs {
  const void* At;
  int64_t ldat;
  const int* idx;
  const double* B;
  int64_t ldb;
  int64_t M, K;
  int Q;
  int64_t kchunk;  // split-K chunk, a multiple of 16
  double* C;       // final result (ksplit == 1) or Q x M partials per chunk (ksplit > 1)
  int64_t ldc;
  const int* kdev;  // if set: K is *kdev (at most g.K) and the gridDim.z chunks split it evenly
};

template <typename XT, int NT>
__global__ __launch_bounds__(256) void k_gemm_f64_rows(F64RowsArgs g) {
  static_assert(F64_RT == 4, "four row tiles: one vector load of four rows per lane");
  typedef F64Frag<XT> FA;
  typedef typename F64Frag<double>::raw b4;
  typedef int i4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t m0 = ((int64_t)blockIdx.x * 4 + wid) * (16 * F64_RT);
  if (m0 >= g.M) return;  // no barrier below: a wave past the last row may leave at once
  const int q0 = (int)blockIdx.y * 16 * NT;
  int64_t K = g.K, kc = g.kchunk;
  if (g.kdev != nullptr) {
    K = min((int64_t)*g.kdev, g.K);
    kc = ((K + gridDim.z - 1) / gridDim.z + 15) / 16 * 16;
  }
  const int64_t kb = (int64_t)blockIdx.z * kc;
  const int64_t ke = min(kb + kc, K);
  const int li = lane & 15;
  const int kk = lane >> 4;
  // rows m0 + 4 li .. + 3 of the transposed design (inside ldat: m0 + 64 <= ldat)
  const XT* ab = (const XT*)g.At + m0 + 4 * li;
  const int* ip = g.idx + kb + 4 * kk;
  const double* bp[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
    bp[t] = g.B + (int64_t)min(q0 + 16 * t + li, g.Q - 1) * g.ldb + kb + 4 * kk;

  f64acc4 acc[F64_RT][NT];
#pragma unroll
  for (int r = 0; r < F64_RT; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[r][t][e] = 0.0;

  const int nsteps = (int)((ke - kb + 15) / 16);
  if (nsteps > 0) {
    // padded steps re-read the last step (valid addresses) and are masked to zero
    const int nsp = (nsteps + F64_PD - 1) / F64_PD * F64_PD;
    const int64_t last = (int64_t)(nsteps - 1) * 16;
    typename FA::raw ra[F64_PD][4];  // [step][sub-step]: elements are the four row tiles
    b4 rb[F64_PD][NT];
    i4 ri[F64_PD];  // row indices of the step F64_PD ahead of the one in ra / rb
#pragma unroll
    for (int d = 0; d < F64_PD; ++d) {
      const int64_t o = min((int64_t)d * 16, last);
      const i4 r0 = *reinterpret_cast<const i4*>(ip + o);
#pragma unroll
      for (int e = 0; e < 4; ++e) ra[d][e] = FA::load(ab + (int64_t)r0[e] * g.ldat);
#pragma unroll
      for (int t = 0; t < NT; ++t) rb[d][t] = *reinterpret_cast<const b4*>(bp[t] + o);
      ri[d] = *reinterpret_cast<const i4*>(ip + min((int64_t)(d + F64_PD) * 16, last));
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int s = 0; s < nsp; s += F64_PD) {
#pragma unroll
      for (int d = 0; d < F64_PD; ++d) {
        __builtin_amdgcn_sched_barrier(0);
        const int64_t kl = kb + (int64_t)(s + d) * 16 + 4 * kk;  // this lane's first k
        double a[F64_RT][4], b[NT][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = kl + e < ke;
#pragma unroll
          for (int r = 0; r < F64_RT; ++r) a[r][e] = ok ? FA::get(ra[d][e], r) : 0.0;
#pragma unroll
          for (int t = 0; t < NT; ++t) b[t][e] = ok ? rb[d][t][e] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int r = 0; r < F64_RT; ++r)
#pragma unroll
            for (int t = 0; t < NT; ++t)
              acc[r][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r][e], b[t][e], acc[r][t], 0, 0, 0);
        const int64_t o = min((int64_t)(s + d + F64_PD) * 16, last);
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[d][e] = FA::load(ab + (int64_t)ri[d][e] * g.ldat);
#pragma unroll
        for (int t = 0; t < NT; ++t) rb[d][t] = *reinterpret_cast<const b4*>(bp[t] + o);
        ri[d] = *reinterpret_cast<const i4*>(ip + min((int64_t)(s + d + 2 * F64_PD) * 16, last));
      }
    }
  }
  // C tile element (i, j) of row tile r sits in lane j + 16 (i % 4), accumulator element i / 4,
  // and is row m0 + 4 i + r
  double* C = g.C + (int64_t)blockIdx.z * g.Q * g.ldc;
#pragma unroll
  for (int r = 0; r < F64_RT; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t m = m0 + 4 * (kk + 4 * e) + r;
        const int q = q0 + 16 * t + li;
        if (m < g.M && q < g.Q) C[(int64_t)q * g.ldc + m] = acc[r][t][e];
      }
}

// C[q][m] = sum over chunks z (in order) of part[z][q][m]
__global__ __launch_bounds__(256) void k_gemm_f64_reduce(const double* __restrict__ part, int ks,
                                                         int Q, int64_t M,
                                                         double* __restrict__ C, int64_t ldc) {
  const int q = blockIdx.y;
  for (int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x; m < M; m += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int z = 0; z < ks; ++z) s += part[((int64_t)z * Q + q) * M + m];
    C[(int64_t)q * ldc + m] = s;
  }
}

}  // namespace cgl

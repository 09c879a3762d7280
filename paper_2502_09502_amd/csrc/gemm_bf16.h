// BF16 MFMA product of the batched engine: C[node][m] = sum_k A[m][k] * B(node, k).
//
//   A: M x K bf16 row-major (the design X~ or its transpose; streamed from HBM once),
//   B: the per-node operands (small, L2 resident), stored in MFMA fragment order (below),
//   C: FP32, node-major (ldc); split-K partials at c_split_stride.
// M is a multiple of the row tile (32 RT), K a multiple of 2 GT_K per chunk, nodes a multiple of
// GT_N.
//
// Workgroup: 32 RT rows of A x 256 nodes, 4 waves; wave w owns nodes [64 w, 64 w + 64) as
// RT x 2 v_mfma_f32_32x32x16_bf16 tiles (rows x nodes), 32 RT accumulators per lane. Three row
// tilings, chosen per product shape by the engine's autotuner: RT = 8 (256 rows, one wave per
// SIMD; the tallest tile reads the least of B from L2, since every row tile reads all of B
// once), RT = 4 (128 rows) and RT = 2 (64 rows): more workgroups for the same rows, so fewer
// k-chunks and fewer partial sums fill the chip, for four times the L2 reads of B at RT = 2
// (two workgroups per CU at RT = 4 would leave too few registers for the prefetch buffers).
// The A tile (32 RT x 64) is
// shared through a two-slot LDS ring (rows of 144 bytes: 9 units of 16 bytes, so that 16 lanes
// reading 16 consecutive rows hit 16 distinct bank groups); each wave's B fragments go straight
// from global memory into registers (each B element is used by exactly one wave of the
// workgroup).
//
// Fragment order of B: the 32 x 16 (nodes x k) fragment that one MFMA consumes is stored as
// 64 lanes x 8 bf16, lane = node % 32 + 32 ((k / 8) % 2), so a wave loads it with one fully
// contiguous 1 KiB access. Fragments are ordered by k-block of 16, then node block of 32.
//
// Latency: vector-memory loads retire in issue order, so a wait for one load also waits for
// every older one. Each k-step's A tile is loaded two steps ahead, right after the previous
// tile of its slot went to LDS, and its B fragments two steps ahead after the step's MFMAs. The
// A fragments of a k-block are read from LDS one k-block ahead of their MFMAs.
#pragma once

#include "common.h"

namespace cgl {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int GT_M = 256;  // the taller row tile (padding unit of the engine's row counts)
constexpr int GT_N = 256;
constexpr int GT_K = 64;
constexpr int GT_RT = GT_M / 32;  // row tiles of 32 per wave in the taller tiling
constexpr int GT_KB = GT_K / 16;  // k-blocks of 16 per k-step
constexpr int GT_LD = GT_K + 8;   // LDS row pitch in bf16 (144 bytes)

// Element offset of B(node, k) in fragment order with nb node blocks of 32.
__device__ __forceinline__ int64_t frag_index(int64_t node, int64_t k, int64_t nb) {
  return (((k >> 4) * nb + (node >> 5)) * 64 + ((node & 31) + 32 * ((k >> 3) & 1))) * 8 + (k & 7);
}

struct GemmArgs {
  const uint16_t* A;
  int64_t lda;
  const uint16_t* B;  // fragment order
  int64_t nb;         // node blocks of 32 in B
  int64_t M, K;
  int64_t kchunk;  // split-K chunk (multiple of 2 GT_K)
  float* C;
  int64_t ldc;
  int64_t c_split_stride;
};

// A tile row segment, as a streaming (non-temporal) load when NT: the caches then do not keep
// the design, whose rows are read once per pass.
template <bool NT>
__device__ __forceinline__ u32x4 load_a16(const uint16_t* p) {
  if (NT) return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return *reinterpret_cast<const u32x4*>(p);
}

// Main loop; leaves this wave's RT x 2 accumulator tiles (row block r, node block c) in acc.
template <int RT, bool NT = false>
__device__ __forceinline__ void gemm_bf16_mainloop(const GemmArgs& g, int64_t m0, int64_t n0,
                                                   int64_t k0, int64_t k1, uint16_t* As,
                                                   floatx16 (&acc)[RT][2]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[r][c][e] = 0.f;
  const int nsteps = (int)((k1 - k0) / GT_K);
  if (nsteps <= 0) return;
  // A loader: thread t moves rows t / 8 + 32 j (j < RT), 16 bytes at k offset (t % 8) * 8
  const int arow = tid >> 3;
  const int ak = (tid & 7) * 8;
  const uint16_t* ag = g.A + (m0 + arow) * g.lda + k0 + ak;
  const int64_t arow_stride = 32 * g.lda;
  // B fragments of node blocks (n0 + 64 wid) / 32 + c, k-block k0 / 16 + GT_KB step + kb
  const int64_t fkb = g.nb * 512;       // elements per k-block of 16
  const int64_t fstep = GT_KB * fkb;    // per k-step
  const uint16_t* bg = g.B + ((k0 >> 4) * g.nb + ((n0 + 64 * wid) >> 5)) * 512 + lane * 8;
  const int fr = lane & 31;
  const int fk = (lane >> 5) * 8;

  // nsteps is even (the caller pads K chunks to 2 GT_K), so the body unrolled over the two LDS
  // slots has no conditionals; prefetches past the end re-read the last step (a valid address;
  // the values are not used).
  u32x4 ra[2][RT];
  bf16x8 rb[2][GT_KB][2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int j = 0; j < RT; ++j)
      ra[d][j] = load_a16<NT>(ag + j * arow_stride + (int64_t)d * GT_K);
    const uint16_t* b = bg + (int64_t)d * fstep;
#pragma unroll
    for (int kb = 0; kb < GT_KB; ++kb)
#pragma unroll
      for (int c = 0; c < 2; ++c) rb[d][kb][c] = *reinterpret_cast<const bf16x8*>(b + kb * fkb + c * 512);
    // issue the groups oldest first, so the in-loop waits see the same order as the steady state
    __builtin_amdgcn_sched_barrier(0);
  }
  const int64_t last = (int64_t)(nsteps - 1);
  for (int s = 0; s < nsteps; s += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      // keep the program order of the groups: the scheduler must not hoist later prefetches
      // above this step's waits
      __builtin_amdgcn_sched_barrier(0);
      uint16_t* slot = As + d * (32 * RT * GT_LD);
#pragma unroll
      for (int j = 0; j < RT; ++j)
        *reinterpret_cast<u32x4*>(slot + (arow + 32 * j) * GT_LD + ak) = ra[d][j];
      __builtin_amdgcn_sched_barrier(0);
      {
        const int64_t st = min((int64_t)(s + d + 2), last);
#pragma unroll
        for (int j = 0; j < RT; ++j)
          ra[d][j] = load_a16<NT>(ag + j * arow_stride + st * GT_K);
      }
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
      bf16x8 af[2][RT];
#pragma unroll
      for (int r = 0; r < RT; ++r)
        af[0][r] = *reinterpret_cast<const bf16x8*>(slot + (r * 32 + fr) * GT_LD + fk);
#pragma unroll
      for (int kb = 0; kb < GT_KB; ++kb) {
        if (kb + 1 < GT_KB) {
#pragma unroll
          for (int r = 0; r < RT; ++r)
            af[(kb + 1) & 1][r] = *reinterpret_cast<const bf16x8*>(
                slot + (r * 32 + fr) * GT_LD + (kb + 1) * 16 + fk);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[kb & 1][r], rb[d][kb][c],
                                                                acc[r][c], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      {
        const int64_t st = min((int64_t)(s + d + 2), last);
        const uint16_t* b = bg + st * fstep;
#pragma unroll
        for (int kb = 0; kb < GT_KB; ++kb)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            rb[d][kb][c] = *reinterpret_cast<const bf16x8*>(b + kb * fkb + c * 512);
      }
    }
  }
}

// =====================================================================================
// The product kernel: the main loop above per (row tile, k-chunk), split-K partials stored
// node-major.
// Element e of lane l in tile c: row i = (e % 4) + 4 (l / 32) + 8 (e / 4), node j = l % 32.
// =====================================================================================
// PASS only names the instantiation (0: X~ (beta - beta_0), 1: X~^T (grad - r_0)) so that
// profiles report the two products separately; RT: row tiles of 32 per wave (8, 4 or 2, above).
//
// 1D grid, XCD-aware: workgroups are dispatched round-robin over the 8 XCDs by linear id, so the
// (row tile, k-chunk) pairs, ordered k-chunk-major, are cut into 8 contiguous ranges and range x
// is given to the ids that land on XCD x. The workgroups of one XCD then share one or two
// k-chunks of B in that XCD's L2. Node tiles (blockIdx.y) are outermost.
//
// bump (optional): the cycle counter, advanced by one thread of the launch; no kernel of the
// launch reads it and the kernels after it see the new value.
// extent (X pass only): the operand extent counters (the pass reads the columns below the larger
// of extent[0] and extent[1]); with bump, extent[2] and extent[3] accumulate the columns read
// (units of 2 GT_K) and the passes.
// The X^T pass streams all of X~^T (larger than the last-level cache) with non-temporal loads,
// which leaves that cache to the X pass's support prefix of X~.
#ifndef CGL_STREAM_XT
#define CGL_STREAM_XT 1
#endif
constexpr bool kStreamXt = CGL_STREAM_XT != 0;
template <int PASS, int RT>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g, int mtiles, int ks, int per_xcd,
                                                   int* bump, int* extent) {
  static_assert(RT == 8 || RT == 4 || RT == 2, "row tilings of 256, 128 and 64 rows");
  __shared__ __attribute__((aligned(16))) uint16_t As[2 * 32 * RT * GT_LD];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int pair = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (pair >= mtiles * ks) return;  // padding of the last range (no barrier reached yet)
  const int z = pair / mtiles;
  const int64_t m0 = (int64_t)(pair % mtiles) * (32 * RT);
  const int64_t n0 = (int64_t)blockIdx.y * GT_N;
  int64_t K = g.K, kc = g.kchunk;
  if (extent != nullptr) {
    // X pass: the operand is zero at positions >= max(extent[0], extent[1]); the ks chunks
    // split that prefix (multiples of 2 GT_K; chunks past it are empty and store zeros)
    const int64_t e = max(extent[0], extent[1]);
    K = min(K, (e + 2 * GT_K - 1) / (2 * GT_K) * (2 * GT_K));
    kc = ((K + ks - 1) / ks + 2 * GT_K - 1) / (2 * GT_K) * (2 * GT_K);
  }
  if (bump != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    *bump += 1;
    if (extent != nullptr) {  // statistics: extents read (units of 2 GT_K columns), passes
      extent[2] += (int)(K / (2 * GT_K));
      extent[3] += 1;
    }
  }
  const int64_t k0 = (int64_t)z * kc;
  const int64_t k1 = min(K, k0 + kc);
  floatx16 acc[RT][2];
  gemm_bf16_mainloop<RT, PASS == 1 && kStreamXt>(g, m0, n0, k0, k1, As, acc);
  float* C = g.C + (int64_t)z * g.c_split_stride;
  const int hi = lane >> 5;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int64_t node = n0 + wid * 64 + c * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t m = m0 + r * 32 + 4 * hi + 8 * q;
        float4 v;
        v.x = acc[r][c][4 * q + 0];
        v.y = acc[r][c][4 * q + 1];
        v.z = acc[r][c][4 * q + 2];
        v.w = acc[r][c][4 * q + 3];
        *reinterpret_cast<float4*>(C + node * g.ldc + m) = v;
      }
  }
}

}  // namespace cgl

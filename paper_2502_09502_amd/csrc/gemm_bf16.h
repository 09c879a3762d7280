// BF16 MFMA product of the batched engine: C[node][m] = sum_k A[m][k] * B(node, k).
//
//   A: M x K bf16 row-major (the design X~ or its transpose; streamed from HBM once),
//   B: the per-node operands (small, L2 resident), stored in MFMA fragment order (below),
//   C: FP32, node-major (ldc); split-K partials at c_split_stride.
// M is a multiple of GT_M, K a multiple of GT_K * GT_PD per chunk, nodes a multiple of GT_N.
//
// Workgroup: 128 rows of A x 256 nodes, 4 waves; wave w owns nodes [64 w, 64 w + 64) as
// 4 x 2 v_mfma_f32_32x32x16_bf16 tiles (rows x nodes). The A tile (128 x 32) is shared through
// a two-slot LDS ring; each wave's B fragments go straight from global memory into registers
// (each B element is used by exactly one wave of the workgroup).
//
// Fragment order of B: the 32 x 16 (nodes x k) fragment that one MFMA consumes is stored as
// 64 lanes x 8 bf16, lane = node % 32 + 32 ((k / 8) % 2), so a wave loads it with one fully
// contiguous 1 KiB access. Fragments are ordered by k-block of 16, then node block of 32.
//
// Latency: vector-memory loads retire in issue order, so a wait for one load also waits for
// every older one. The A tile of a k-step (HBM) is loaded GT_PD steps ahead of its use and the
// B fragments (L2 resident) GT_PDB steps ahead, B first within a step's group, so that a wait
// only concerns the oldest loads. The eight A fragments of a step are read from LDS in one
// group before its MFMAs: the LDS latency is paid once per step rather than once per MFMA pair
// (and the B registers freed by the shorter B prefetch hold them).
#pragma once

#include "common.h"

namespace cgl {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int GT_M = 128;
constexpr int GT_N = 256;
constexpr int GT_K = 32;
constexpr int GT_RT = GT_M / 32;  // row tiles per wave
constexpr int GT_LD = GT_K + 8;   // LDS row pitch in bf16 (80 bytes)
constexpr int GT_PD = 4;          // A k-steps in flight (even: the LDS slot of step s is s & 1)
constexpr int GT_PDB = 2;         // B k-steps in flight (divides GT_PD)

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
  int64_t kchunk;  // split-K chunk (multiple of GT_K * GT_PD)
  float* C;
  int64_t ldc;
  int64_t c_split_stride;
};

// Main loop; leaves this wave's GT_RT x 2 accumulator tiles (row block r, node block c) in acc.
__device__ __forceinline__ void gemm_bf16_mainloop(const GemmArgs& g, int64_t m0, int64_t n0,
                                                   int64_t k0, int64_t k1, uint16_t* As,
                                                   floatx16 (&acc)[GT_RT][2]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
#pragma unroll
  for (int r = 0; r < GT_RT; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[r][c][e] = 0.f;
  const int nsteps = (int)((k1 - k0) / GT_K);
  if (nsteps <= 0) return;
  // A loader: thread t moves 2 x 16 bytes: rows t / 4 and t / 4 + 64, k offset (t % 4) * 8
  const int arow = tid >> 2;
  const int ak = (tid & 3) * 8;
  const uint16_t* ag = g.A + (m0 + arow) * g.lda + k0 + ak;
  const int64_t ag_hi = 64 * g.lda;
  // B fragments of node blocks (n0 + 64 wid) / 32 + c, k-block k0 / 16 + 2 step + ks
  const int64_t fstep = 2 * g.nb * 512;  // elements per k-step of 32
  const int64_t fks = g.nb * 512;
  const uint16_t* bg = g.B + ((k0 >> 4) * g.nb + ((n0 + 64 * wid) >> 5)) * 512 + lane * 8;
  const int fr = lane & 31;
  const int fk = (lane >> 5) * 8;

  // nsteps is a multiple of GT_PD (the caller pads K chunks to GT_K * GT_PD), so the unrolled
  // body below has no conditionals and the register arrays stay in registers; prefetches past
  // the end re-read the last step (a valid address; the values are not used).
  u32x4 ra[GT_PD][2];
  bf16x8 rb[GT_PDB][2][2];
#pragma unroll
  for (int d = 0; d < GT_PD; ++d) {
    if (d < GT_PDB) {
      const uint16_t* b = bg + (int64_t)d * fstep;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int c = 0; c < 2; ++c) rb[d][c][ks] = *reinterpret_cast<const bf16x8*>(b + ks * fks + c * 512);
    }
    const int64_t o = (int64_t)d * GT_K;
    ra[d][0] = *reinterpret_cast<const u32x4*>(ag + o);
    ra[d][1] = *reinterpret_cast<const u32x4*>(ag + ag_hi + o);
    // issue the groups oldest first, so the in-loop waits see the same order as the steady state
    __builtin_amdgcn_sched_barrier(0);
  }
  const int64_t last = (int64_t)(nsteps - 1);
  for (int s = 0; s < nsteps; s += GT_PD) {
#pragma unroll
    for (int d = 0; d < GT_PD; ++d) {
      // keep the program order of the groups: the scheduler must not hoist later prefetches
      // above this step's wait (that would turn the rolling pipeline into a per-block one)
      __builtin_amdgcn_sched_barrier(0);
      uint16_t* slot = As + (d & 1) * (GT_M * GT_LD);
      *reinterpret_cast<u32x4*>(slot + arow * GT_LD + ak) = ra[d][0];
      *reinterpret_cast<u32x4*>(slot + (arow + 64) * GT_LD + ak) = ra[d][1];
      __syncthreads();
      bf16x8 af[2][GT_RT];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int r = 0; r < GT_RT; ++r)
          af[ks][r] = *reinterpret_cast<const bf16x8*>(slot + (r * 32 + fr) * GT_LD + ks * 16 + fk);
      __builtin_amdgcn_sched_barrier(0);
      const int db = d % GT_PDB;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
        for (int r = 0; r < GT_RT; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[ks][r], rb[db][c][ks], acc[r][c],
                                                                0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      {
        const int64_t st = min((int64_t)(s + d + GT_PDB), last);
        const uint16_t* b = bg + st * fstep;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            rb[db][c][ks] = *reinterpret_cast<const bf16x8*>(b + ks * fks + c * 512);
      }
      const int64_t st = min((int64_t)(s + d + GT_PD), last);
      ra[d][0] = *reinterpret_cast<const u32x4*>(ag + st * GT_K);
      ra[d][1] = *reinterpret_cast<const u32x4*>(ag + ag_hi + st * GT_K);
    }
  }
}

}  // namespace cgl

// Batched mixed-precision engine kernels.
//
// S node slots share one design X. Each slot iterates Alg. 3 around an FP64 base point beta_0
// with FP64 quantities u_0 = X beta_0, r_0 = grad f(u_0), H_0 = X^T r_0. The two products of an
// iteration are corrections to that base, computed for all slots at once on MFMA with BF16
// operands and FP32 accumulation:
//
//   dU = X~ bf16(beta^{t+1} - beta_0)           (X pass; S x n)
//   dH = X~^T bf16(grad f(u_gamma) - r_0)       (X^T pass; S x p), u_gamma = u_0 + dU_gamma
//
// so grad F(gamma) = H_0 + dH and f(X beta^{t+1}) = f(u_0 + dU). X~ is the BF16 copy of X (equal
// to X when X is stored in BF16). Errors of the BF16 operands are relative to the size of the
// correction, which shrinks as the iterate approaches the base; the base is re-centred in FP64
// (and the bound certified, Sec. 3.4) when the working-precision gap stops improving.
//
// One iteration (cycle) for every active slot: k_gemm_x (split-K; it also advances the cycle
// counter) -> k_mixed_loss (loss partials and the residual operand for both outcomes of the
// restart test) -> k_mixed_decide (restart test; the chosen operand into gop) -> k_gemm_xt
// (split-K) -> k_mixed_node (prox; commits the restart test).
#include <limits.h>

#include <algorithm>

#include <hip/hip_ext.h>

#include "common.h"
#include "kernels.h"
#include "gemm_bf16.h"
#include "gemm_f64.h"
#include "losses.h"
#include "mixed.h"
#include "prox.h"
#include "solver.h"

namespace cgl {

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4;



// A slot advances while it holds a node that is not finished and has iterations left (a slot at
// its cap waits for the certification that ends it).
__device__ __forceinline__ bool slot_running(const NodeDev* st) {
  return st->active != 0 && st->done == 0 && st->need_base == 0 && st->iter < st->max_iter;
}

// Momentum coefficient of Alg. 3 for the counter phi. The loss kernel's operand candidates and
// the decision kernel's stored coefficient both come from here, so the two agree bit for bit.
__device__ __forceinline__ double momentum_coef(double phi) { return phi / (phi + 3.0); }

// =====================================================================================
// One pass over each slot's rows after the X pass (grid: (chunks, slots); 256 threads):
// * dU^{t+1} = the sum of the X-pass split-K partials, into the ring slot of this cycle;
// * the loss terms f_i(u_0 + dU) summed per chunk (and their rounding scale, for the margin of
//   the restart test);
// * the residual operand of the X^T pass, G = bf16(grad f(u_gamma) - r_0) with u_gamma = u_0 +
//   dU^{t+1} + c (dU^{t+1} - dU^t), and on the dual monitor's iterations the F*(-zeta) partial
//   sums at u_gamma (zeta = -grad f(u_gamma)).
// The momentum coefficient c depends on the restart test (Alg. 3), which needs f(X beta^{t+1})
// summed over every chunk. It takes one of two values that are known beforehand: c_r = 1/4 after
// a restart (phi = 1), c_k for phi + 1 otherwise (phi itself while the momentum is not yet
// primed). The kernel therefore writes G and the F* partials for both: gop (fragment order) and
// fpart set 0 for c_k, gop_r (slot-major) and set 1 for c_r (only c_k when no restart is
// possible this cycle: unprimed, or the first cycle after a rebase). k_mixed_decide takes the
// test and leaves the chosen operand in gop; the node kernel reads the chosen F* partials.
//
// In the first cycle after a re-centre that kept the momentum (rebase), the product of this
// cycle is X~ bf16(beta^{t+1} - beta_0') against the previous base beta_0', and beta^{t+1} is the
// new base: dU^{t+1} = 0 and the previous correction becomes X~ bf16(beta^t - beta_0') minus this
// product, i.e. X (beta^t - beta^{t+1}) with the rounding of an ordinary cycle's difference.
// =====================================================================================
// LS: the instantiation for the least-squares slots (the other serves the other losses; an engine
// launches the ones its problems need). The least-squares code alone needs far fewer registers
// than the FP64 transcendental work of the other losses; its kernel asks for 6 waves per SIMD
// (it fits 8 without spills), so more waves keep loads in flight.
template <bool LS>
__device__ __forceinline__ void mixed_loss_body(const MixedDev& md) {
  __shared__ double red[4][4];
  // the X pass of this cycle has read the operand extent: its counter restarts for cycle + 2
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) md.keff[*md.cycle & 1] = 0;
  const int slot = blockIdx.y;
  const NodeDev* st = md.st + slot;
  if (!slot_running(st)) return;
  const MemberDev& mb = md.mem[st->member];
  const int loss = mb.loss;
  if ((loss == LOSS_LS) != LS) return;
  const double* yv = mb.y;
  const int cyc = *md.cycle;
  const bool rebase = st->rebase != 0;
  // the two candidates of the momentum coefficient, and whether the node kernel of this cycle
  // runs the dual monitor (uniform over the block)
  const bool can_restart = st->primed != 0 && !rebase;
  const double ck = momentum_coef(st->primed != 0 ? st->phi + 1.0 : st->phi);
  const double cr = momentum_coef(1.0);
  const bool check = (st->iter % st->check_every) == 0;
  float* dun = md.dU + (int64_t)(cyc & 1) * md.dU_ring + (int64_t)slot * md.n_pad;
  float* duo = md.dU + (int64_t)((cyc + 1) & 1) * md.dU_ring + (int64_t)slot * md.n_pad;
  const int64_t i0 = (int64_t)blockIdx.x * md.rchunk;
  const int64_t i1 = min(md.n_pad, i0 + md.rchunk);
  // strays of the operand: X~ column j is row j of X~^T; each thread sums them for 8 consecutive
  // rows of the chunk (16-byte loads), in list order. The list goes through LDS first and the
  // rows are loaded eight strays at a time: one slot's strays are a chain of dependent loads
  // otherwise, which sets the kernel's time when few slots run.
  const int ns = md.sn[slot];
  __shared__ float sdu[kLossChunk];
  __shared__ int sjs[kStrayCap];
  __shared__ float svs[kStrayCap];
  if (ns > 0) {  // uniform over the block
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    if (threadIdx.x < ns) {
      sjs[threadIdx.x] = md.sj[(int64_t)slot * kStrayCap + threadIdx.x];
      svs[threadIdx.x] = md.sv[(int64_t)slot * kStrayCap + threadIdx.x];
    }
    __syncthreads();
    const int64_t r8 = 8 * (int64_t)threadIdx.x;
    if (i0 + r8 < i1) {
      const uint16_t* xr = md.Xbt + i0 + r8;
      float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      auto add = [&](const u32x4& x, float v) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
          a[c] += bf16_to_float((uint16_t)((x[c >> 1] >> (16 * (c & 1))) & 0xffffu)) * v;
      };
      int e = 0;
      for (; e + 8 <= ns; e += 8) {
        u32x4 x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          x[q] = *reinterpret_cast<const u32x4*>(xr + (int64_t)sjs[e + q] * md.n_pad);
#pragma unroll
        for (int q = 0; q < 8; ++q) add(x[q], svs[e + q]);
      }
      for (; e < ns; ++e)
        add(*reinterpret_cast<const u32x4*>(xr + (int64_t)sjs[e] * md.n_pad), svs[e]);
#pragma unroll
      for (int c = 0; c < 8; ++c) sdu[r8 + c] = a[c];
    }
    __syncthreads();
  }
  // four consecutive rows per thread and step (16-byte loads and stores, 8-byte operand stores;
  // n_pad and the chunk bounds are multiples of 256)
  double ls = 0.0, nz = 0.0, fk = 0.0, fr = 0.0;
  const bool noise = md.restart_slack > 0.0;  // uniform: a launch argument
  const float* dup = md.dUp + (int64_t)slot * md.n_pad;
  const int64_t nbk = md.S_pad >> 5;
  for (int64_t i = i0 + 4 * (int64_t)threadIdx.x; i < i1; i += 4 * 256) {
    float4 du = *reinterpret_cast<const float4*>(dup + i);
    for (int q = 1; q < md.ksx; ++q) {
      const float4 t = *reinterpret_cast<const float4*>(dup + (int64_t)q * md.dUp_split + i);
      du.x += t.x;
      du.y += t.y;
      du.z += t.z;
      du.w += t.w;
    }
    if (ns > 0) {
      du.x += sdu[i - i0];
      du.y += sdu[i - i0 + 1];
      du.z += sdu[i - i0 + 2];
      du.w += sdu[i - i0 + 3];
    }
    float4 o = *reinterpret_cast<const float4*>(duo + i);  // dU^t
    if (rebase) {
      o.x -= du.x;
      o.y -= du.y;
      o.z -= du.z;
      o.w -= du.w;
      *reinterpret_cast<float4*>(duo + i) = o;
      du = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    *reinterpret_cast<float4*>(dun + i) = du;
    const float dv[4] = {du.x, du.y, du.z, du.w}, ov[4] = {o.x, o.y, o.z, o.w};
    uint16_t gk[4] = {0, 0, 0, 0}, gr[4] = {0, 0, 0, 0};
    if constexpr (LS) {
      const float4 e4 = *reinterpret_cast<const float4*>(md.e0f + (int64_t)slot * md.n_pad + i);
      const float ev[4] = {e4.x, e4.y, e4.z, e4.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (i + c < md.n) {
          const double e = (double)ev[c] + (double)dv[c];  // u - y
          ls += e * e;
          if (noise) {
            const double t = 2.0 * e * (double)dv[c];
            nz += t * t;
          }
          const double y = yv[i + c];
          // gamma's correction for each candidate; r = 2 (u_gamma - y); F*(-zeta) at zeta = -r
          // is ||zeta||^2 / 4 - y.zeta
          const double dgk = (double)dv[c] + ck * ((double)dv[c] - (double)ov[c]);
          gk[c] = float_to_bf16((float)(2.0 * dgk));
          if (check) {
            const double r = 2.0 * ((double)ev[c] + dgk);
            fk += 0.25 * r * r + y * r;
          }
          if (can_restart) {
            const double dgr = (double)dv[c] + cr * ((double)dv[c] - (double)ov[c]);
            gr[c] = float_to_bf16((float)(2.0 * dgr));
            if (check) {
              const double r = 2.0 * ((double)ev[c] + dgr);
              fr += 0.25 * r * r + y * r;
            }
          }
        }
      }
    } else {  // base0 holds u_0, base1 holds r_0 = grad f(u_0)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (i + c < md.n) {
          const double u0 = md.base0[(int64_t)slot * md.n_pad + i + c];
          const double r0 = md.base1[(int64_t)slot * md.n_pad + i + c];
          const double y = yv[i + c];
          const double u = u0 + (double)dv[c];
          ls += loss_val(loss, u, y);
          if (noise) {
            const double t = loss_grad(loss, u, y) * (double)dv[c];
            nz += t * t;
          }
          const double ugk = u0 + ((double)dv[c] + ck * ((double)dv[c] - (double)ov[c]));
          gk[c] = float_to_bf16((float)(loss_grad(loss, ugk, y) - r0));
          if (check) fk += fstar_term(loss, ugk, y);
          if (can_restart) {
            const double ugr = u0 + ((double)dv[c] + cr * ((double)dv[c] - (double)ov[c]));
            gr[c] = float_to_bf16((float)(loss_grad(loss, ugr, y) - r0));
            if (check) fr += fstar_term(loss, ugr, y);
          }
        }
      }
    }
    // rows i .. i + 3 are consecutive within one 8-row group of the fragment layout
    const int64_t f = frag_index(slot, i, nbk);
    uint2 w;
    w.x = (uint32_t)gk[0] | ((uint32_t)gk[1] << 16);
    w.y = (uint32_t)gk[2] | ((uint32_t)gk[3] << 16);
    *reinterpret_cast<uint2*>(md.gop + f) = w;
    if (can_restart) {  // slot-major: only the decision kernel reads it
      w.x = (uint32_t)gr[0] | ((uint32_t)gr[1] << 16);
      w.y = (uint32_t)gr[2] | ((uint32_t)gr[3] << 16);
      *reinterpret_cast<uint2*>(md.gop_r + (int64_t)slot * md.n_pad + i) = w;
    }
  }
  // the four sums of the block in one pass: per wave, then over the waves
  const double v4[4] = {ls, nz, fk, fr};
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double t = wave_sum(v4[v]);
    if (lane == 0) red[v][wid] = t;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int v = threadIdx.x;
    const double t = (red[v][0] + red[v][1]) + (red[v][2] + red[v][3]);
    const int64_t b = (int64_t)slot * md.nrt + blockIdx.x;
    if (v == 0) md.lpart[b] = t;
    // the rounding scale of this chunk's loss terms: each dU_i carries a relative error of
    // about 2^-9 (BF16 operand), which moves f by about f_i'(u) dU_i 2^-9
    else if (v == 1 && noise) md.npart[b] = t;
    else if (v == 2 && check) md.fpart[((int64_t)slot * 2) * md.nrt + blockIdx.x] = t;
    else if (v == 3 && check && can_restart)
      md.fpart[((int64_t)slot * 2 + 1) * md.nrt + blockIdx.x] = t;
  }
}

template <bool LS>
__global__ void k_mixed_loss(MixedDev md);
template <>
__global__ __launch_bounds__(256, 6) void k_mixed_loss<true>(MixedDev md) {
  mixed_loss_body<true>(md);
}
template <>
__global__ __launch_bounds__(256) void k_mixed_loss<false>(MixedDev md) {
  mixed_loss_body<false>(md);
}

// =====================================================================================
// Restart test of Alg. 3 for every running slot: L^{t+1} = f(X beta^{t+1}) + 2 lambda2
// g(beta^{t+1}) from the loss kernel's partials (in chunk order), against L^t plus the rounding
// margin. Block 0 of a slot stores the momentum coefficient and the outcome, which the node
// kernel commits, and gsel (1 after a restart: the node kernel then reads F* partial set 1).
// After a restart every block copies its share of the slot's restart operand (gop_r) over gop,
// so that the X^T pass reads one buffer (the two candidates of a node block in separate buffers
// would double the pass's B traffic through L2). Every block evaluates the test from the same
// partials with the same instructions, so they agree. grid: (kDecideBlocks, slots); 256 threads.
// =====================================================================================
constexpr int kDecideBlocks = 4;

__global__ __launch_bounds__(256) void k_mixed_decide(MixedDev md) {
  __shared__ int sel_s;
  const int slot = blockIdx.y;
  const NodeDev* st = md.st + slot;
  if (threadIdx.x < 64) {
    // the partials and the slot's state are loaded together (neither address depends on the
    // other); the sums run across the wave in a fixed order, so every block gets the same values
    const double* lp = md.lpart + (int64_t)slot * md.nrt;
    const double* np = md.npart + (int64_t)slot * md.nrt;
    const bool noise = md.restart_slack > 0.0;
    double a = 0.0, nz = 0.0;
    for (int i = threadIdx.x; i < md.nrt; i += 64) {
      a += lp[i];
      if (noise) nz += np[i];
    }
    const bool run = slot_running(st);
    const int primed = st->primed, rebase = st->rebase, restarts = st->restarts;
    const double phi = st->phi, L_prev = st->L_prev, bsq = st->bsq_new, gnew = st->g_new;
    const int mi = st->member;  // read before the slot is known to run: kept in the table
    const MemberDev& mb = md.mem[(unsigned)mi < (unsigned)kMaxMembers ? mi : 0];
    const double shift = mb.shift, lam2 = mb.lam2;
    a = wave_sum(a);
    nz = wave_sum(nz);
    if (threadIdx.x == 0) {
      int sel = -1;  // not running: nothing to decide
      if (run) {
        // rounding margin of the working objective (zero: Alg. 3's plain comparison)
        const double margin = md.restart_slack * 0x1p-9 * sqrt(nz);
        const double Lnew = a - shift * bsq + 2.0 * (lam2 + shift) * gnew;
        double phin = phi;
        int primedn = primed, restartsn = restarts;
        sel = 0;
        if (!primed) {
          primedn = 1;
        } else if (rebase) {
          // L^t was evaluated against the previous base: the momentum runs on untested
          phin += 1.0;
        } else if (Lnew >= L_prev + margin) {
          phin = 1.0;
          restartsn += 1;
          sel = 1;
        } else {
          phin += 1.0;
        }
        if (blockIdx.x == 0) {
          NodeDev* sw = md.st + slot;
          sw->c = momentum_coef(phin);
          sw->rs_phi = phin;
          sw->rs_L = Lnew;
          sw->rs_primed = primedn;
          sw->rs_restarts = restartsn;
          md.gsel[slot] = sel;
        }
      }
      sel_s = sel;
    }
  }
  __syncthreads();
  if (sel_s <= 0) return;
  // rows 8t .. 8t + 7 of the slot (16 bytes of gop_r, slot-major) are one segment of the
  // fragment order: k-block t / 2, lane slot % 32 (t even) or slot % 32 + 32 (t odd) of the
  // slot's node block
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const int64_t nb = md.S_pad >> 5;
  const int64_t nseg = md.n_pad >> 3;
  const uint16_t* src = md.gop_r + (int64_t)slot * md.n_pad;
  // four segments per thread and round: their loads are issued before any of the stores (one
  // load latency per round rather than one per segment)
  const int64_t step = (int64_t)gridDim.x * 256;
  for (int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x; t0 < nseg; t0 += 4 * step) {
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (t0 + k * step < nseg) v[k] = *reinterpret_cast<const u32x4*>(src + 8 * (t0 + k * step));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t t = t0 + k * step;
      if (t < nseg)
        *reinterpret_cast<u32x4*>(md.gop + ((t >> 1) * nb + (slot >> 5)) * 512 +
                                  ((slot & 31) + 32 * (t & 1)) * 8) = v[k];
    }
  }
}

// =====================================================================================
// Per-slot gradient step, prox, operand update and dual monitor. One 1024-thread workgroup
// per slot.
// =====================================================================================
template <int E>
__global__ __launch_bounds__(1024) void k_mixed_node(MixedDev md) {
  __shared__ ProxSmem sm;
  const int slot = blockIdx.x;
  NodeDev* st = md.st + slot;
  if (!slot_running(st)) return;
  const MemberDev& mb = md.mem[st->member];
  const double mM = mb.M, mrho = mb.rho;
  const int cyc = *md.cycle;
  const int64_t p = md.p;
  const double* bt1 = md.bring + (int64_t)(cyc % 3) * md.bring_stride + (int64_t)slot * md.ldp;
  const double* bt0 =
      md.bring + (int64_t)((cyc + 2) % 3) * md.bring_stride + (int64_t)slot * md.ldp;
  double* bout = md.bring + (int64_t)((cyc + 1) % 3) * md.bring_stride + (int64_t)slot * md.ldp;
  const double* H0 = md.H0 + (int64_t)slot * md.ldp;
  const double* b0 = md.beta0 + (int64_t)slot * md.ldp;
  const uint8_t* cl = md.cls + (int64_t)slot * md.ldp;
  if (threadIdx.x == 0) {  // commit the restart test of this cycle
    st->phi = st->rs_phi;
    st->primed = st->rs_primed;
    st->restarts = st->rs_restarts;
    st->L_prev = st->rs_L;
    st->L_work = st->rs_L;
    if (st->rs_L < st->P_best) st->P_best = st->rs_L;  // working-precision best (monitor only)
    st->rebase = 0;  // read by the loss and decision kernels of this cycle only
  }
  const double c = st->c;
  const double invL = 1.0 / mb.L;
  const int iter = st->iter;
  const bool check = (iter % st->check_every) == 0;
  // read ahead (their latency is spent on the loads of H): the winners of this slot's last two
  // selections (where the registers allow), and the F* partials of the loss kernel at the chosen
  // gamma (summed per wave below; read only when the dual monitor runs)
  constexpr bool kAhead = E <= 12;
  int* const rtop = md.prevtop + (int64_t)slot * 65;
  int* const rhead = md.prevhead + (int64_t)slot * 65;
  WarmPrev wtop{rtop, -1, 0}, whead{rhead, -1, 0};
  if (kAhead) {
    wtop = warm_prev(rtop);
    whead = warm_prev(rhead);
  }
  double fpre = 0.0;
  if (check) {
    const double* fp = md.fpart + ((int64_t)slot * 2 + (md.gsel[slot] != 0)) * md.nrt;
    for (int i = threadIdx.x; i < md.nrt; i += blockDim.x) fpre += fp[i];
  }
  // H at gamma (FP64 base + BF16-product corrections) into the per-thread value slice
  __shared__ double vbuf[ProxVals<E>::nl * kProxThreads];
  ProxVals<E> pv;
  pv.sl = vbuf;
  uint64_t cb = 0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
    double h = 0.0;
    int cs = CLS_PAD;
    if (j < p) {
      h = H0[j];
      cs = cl[j];
    }
    pv.set(s, h);
    cb |= (uint64_t)cs << (2 * s);
  }
  // split-K partials two slabs at a time while the registers allow it (E <= 12): both slabs'
  // loads are in flight together, and each value still takes the slabs in order (same
  // summation order as one slab at a time)
  int q = 0;
  for (; E <= 12 && q + 2 <= md.ksplit; q += 2) {
    const float* dq0 = md.dH + (int64_t)q * md.dH_split + (int64_t)slot * md.ldp;
    const float* dq1 = dq0 + md.dH_split;
    float a0[E], a1[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
      a0[s] = j < p ? dq0[j] : 0.f;
      a1[s] = j < p ? dq1[j] : 0.f;
    }
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
      if (j < p) pv.set(s, (pv.get(s) + (double)a0[s]) + (double)a1[s]);
    }
  }
  for (; q < md.ksplit; ++q) {
    const float* dq = md.dH + (int64_t)q * md.dH_split + (int64_t)slot * md.ldp;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
      if (j < p) pv.set(s, pv.get(s) + (double)dq[j]);
    }
  }
  fpre = wave_sum(fpre);
  if ((threadIdx.x & 63) == 0) sm.fsw[threadIdx.x >> 6] = fpre;  // read after later barriers
  // eigen-perspective shift: the gradient at gamma is X^T grad f(X gamma) - 2 s gamma, and the
  // bound gains s ||gamma||^2 (uniform branch: the shift is a launch argument)
  const double shift = mb.shift;
  const double two_le = 2.0 * (mb.lam2 + shift);
  double gsq = 0.0;
  if (shift != 0.0) {
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
      if (j < p) {
        const double x1 = bt1[j];
        const double gam = x1 + c * (x1 - bt0[j]);
        pv.set(s, pv.get(s) - 2.0 * shift * gam);
        gsq += gam * gam;
      }
    }
    gsq = bsum(gsq, sm);
  }
  // dual monitor at gamma: D = -F*(-zeta) - 2 lambda2 g_node*(-grad F(gamma) / (2 lambda2))
  // element-indexed view of the LDS slice for the warm-started selections
  const double* slice = ProxVals<E>::lds ? vbuf : nullptr;
  double gs = 0.0;
  if (check)
    gs = gstar_node<E>([&](int s) { return fabs(pv.get(s)); }, two_le, cb, st->kp,
                       st->nfree, mM, sm, slice, kAhead ? wtop : warm_prev(rtop));
  // gradient step w = gamma - H / L; the slice then holds u = rho |w|, the signs a mask
  uint32_t neg = 0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
    double w = 0.0;
    if (j < p) {
      const double x1 = bt1[j];
      const double gam = x1 + c * (x1 - bt0[j]);
      w = gam - pv.get(s) * invL;
    }
    neg |= (w < 0.0 ? 1u : 0u) << s;
    pv.set(s, mrho * fabs(w));
  }
  const int64_t nbk = md.S_pad >> 5;
  // operand extent (LDS: nothing extra stays live through the prox)
  __shared__ int ext_s;
  if (threadIdx.x == 0) ext_s = 0;
  __syncthreads();
  // the prox hands each beta_j back into the value slice (its u is not read again)
  double bsq = 0.0;
  const ProxOut po = node_prox<E>(
      [&](int s) { return pv.get(s); }, neg, cb, st->kp, st->nfree, mrho, mM, st->vstar,
      [&](int s, double b) {
        bsq += b * b;
        pv.set(s, b);
      },
      sm, slice, kAhead ? whead : warm_prev(rhead));
  // the new iterate and its operand entries, in groups whose loads of beta_0 and of the column
  // positions are all issued before the group's stores (groups of 4 where registers are short)
  constexpr int G = E <= 12 ? E : 4;
#pragma unroll
  for (int s0 = 0; s0 < E; s0 += G) {
    double b0v[G];
    int posv[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t j = (int64_t)(s0 + g) * kProxThreads + threadIdx.x;
      b0v[g] = 0.0;
      posv[g] = 0;
      if (s0 + g < E && j < p) {
        b0v[g] = b0[j];
        posv[g] = md.pinv[j];
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t j = (int64_t)(s0 + g) * kProxThreads + threadIdx.x;
      if (s0 + g < E && j < p) {
        const double b = pv.get(s0 + g);
        bout[j] = b;
        const uint16_t d = float_to_bf16((float)(b - b0v[g]));
        md.dop[frag_index(slot, posv[g], nbk)] = d;
        if ((d & 0x7fffu) != 0) atomicMax(&ext_s, posv[g] + 1);
      }
    }
  }
  __syncthreads();
  // Entries past the support prefix leave the operand as strays, in position order, when there
  // are at most kStrayCap of them; otherwise they all stay and the extent covers them (their
  // columns are read by the X pass then, so strays would only add reads). Two passes over the
  // operand stores of the whole block (ordered by the barrier above): count per thread,
  // exclusive scan, assign.
  const int pfx = *md.pfx;
  const int ext_all = ext_s;
  int ext = min(ext_all, pfx);
  int ns = 0;
  if (ext_all > pfx) {  // uniform over the block
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const int ubeg = (pfx & ~7) + 8 * (int)threadIdx.x;
    auto late = [&](int u8, const u32x4& v, int e) {
      const int u = u8 + e;
      const uint16_t d = (uint16_t)((v[e >> 1] >> (16 * (e & 1))) & 0xffffu);
      return u >= pfx && u < ext_all && (d & 0x7fffu) != 0;
    };
    int cnt = 0;
    for (int u8 = ubeg; u8 < ext_all; u8 += 8 * kProxThreads) {
      const u32x4 v = *reinterpret_cast<const u32x4*>(md.dop + frag_index(slot, u8, nbk));
      for (int e = 0; e < 8; ++e) cnt += late(u8, v, e) ? 1 : 0;
    }
    // exclusive scan of cnt in thread order (groups of one stride round are in position order
    // across threads, and the rounds are in order)
    __shared__ int wsum[kProxThreads / 64];
    int incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(incl, off, 64);
      if ((threadIdx.x & 63) >= off) incl += o;
    }
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    int base = 0, total = 0;
    for (int w = 0; w < kProxThreads / 64; ++w) {
      if (w < (int)(threadIdx.x >> 6)) base += wsum[w];
      total += wsum[w];
    }
    int idx = base + incl - cnt;
    ns = total <= kStrayCap ? total : 0;
    for (int u8 = ubeg; u8 < ext_all && cnt > 0 && ns > 0; u8 += 8 * kProxThreads) {
      uint16_t* g8 = md.dop + frag_index(slot, u8, nbk);
      const u32x4 v = *reinterpret_cast<const u32x4*>(g8);
      for (int e = 0; e < 8; ++e) {
        if (!late(u8, v, e)) continue;
        const int u = u8 + e;
        md.sj[(int64_t)slot * kStrayCap + idx] = md.perm[u];
        md.sv[(int64_t)slot * kStrayCap + idx] =
            bf16_to_float((uint16_t)((v[e >> 1] >> (16 * (e & 1))) & 0xffffu));
        g8[e] = 0;
        ++idx;
      }
    }
    if (ns == 0) ext = ext_all;
  }
  if (threadIdx.x == 0 && ext > 0) atomicMax(md.keff + ((cyc + 1) & 1), ext);
  if (threadIdx.x == 0) md.sn[slot] = ns;
  double fs = 0.0;
  if (check) {
#pragma unroll
    for (int w = 0; w < kProxWaves; ++w) fs += sm.fsw[w];
  }
  if (shift != 0.0) bsq = bsum(bsq, sm);
  if (threadIdx.x == 0) {
    st->g_new = po.gval;
    st->bsq_new = shift != 0.0 ? bsq : 0.0;
    st->vstar = po.vstar;
    if (check) {
      const double D = -fs - two_le * gs + shift * gsq;
      if (D > st->D_best) st->D_best = D;  // working-precision monitor
    }
    const double Pw = st->P_best, Dw = st->D_best;
    const double mgap = (Pw - Dw) / fmax(fabs(Pw), 1.0);
    if (!(Pw == Pw) || !(po.gval == po.gval)) {
      st->status = 3;  // NUMERIC
      st->done = 1;
    }
    if (mgap < 0.5 * st->mgap_ref) {
      st->mgap_ref = mgap;
      st->since_improve = 0;
    } else {
      st->since_improve += 1;
    }
    st->since_recentre += 1;
    if (mgap <= md.cert_gap * st->tol ||
        (st->since_improve >= md.stall_cycles && st->since_recentre >= md.stall_cycles) ||
        iter + 1 >= st->max_iter) {
      st->want_cert = 1;
    }
    st->iter = iter + 1;
    st->last_ring = (cyc + 1) % 3;
  }
}

// =====================================================================================
// Native-precision transposed copy of X for the FP64 X^T products of certification
// (BF16 designs use the BF16 transpose, which is exact for them).
// =====================================================================================

template <typename XT>
__global__ __launch_bounds__(256) void k_transpose(const XT* __restrict__ X, int64_t ldx, int64_t n,
                                                   int64_t p, int64_t n_pad, XT* __restrict__ Xt) {
  __shared__ XT tile[32][33];
  const int64_t j0 = (int64_t)blockIdx.x * 32, i0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, j = j0 + tx;
    tile[r][tx] = (i < n && j < p) ? X[i * ldx + j] : (XT)0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + r, i = i0 + tx;
    if (j < p && i < n_pad) Xt[j * n_pad + i] = tile[tx][r];
  }
}

// =====================================================================================
// Certification / re-centring helpers
// =====================================================================================

// B64[q][j] = latest iterate of slot list[q] (ring slot cycle % 3); flag[j] = 1 where some
// gathered iterate is nonzero (every writer stores the same value; the flags start at zero).
__global__ __launch_bounds__(256) void k_cert_gather(MixedDev md, const int* list, int nq,
                                                     double* B64, uint8_t* flag) {
  const int q = blockIdx.y;
  if (q >= nq) return;
  const int slot = list[q];
  const int ring = md.st[slot].last_ring;
  const double* src = md.bring + (int64_t)ring * md.bring_stride + (int64_t)slot * md.ldp;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < md.ldp; j += (int64_t)gridDim.x * 256) {
    const double v = src[j];
    B64[(int64_t)q * md.ldp + j] = v;
    if (v != 0.0 && j < md.p) flag[j] = 1;
  }
}

// The union of the gathered supports as a list: idx[0 .. K) = the flagged coordinates in
// increasing order, idx[K .. K rounded up to 16) = 0, *count = K; the flags are cleared for the
// next round. One workgroup.
__global__ __launch_bounds__(1024) void k_cert_support(uint8_t* flag, int64_t p, int* idx,
                                                       int* count) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int64_t per = (p + 1023) / 1024;
  const int64_t j0 = min((int64_t)t * per, p), j1 = min(j0 + per, p);
  int c = 0;
  for (int64_t j = j0; j < j1; ++j) c += flag[j] != 0;
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int o = part[t] - c;
  for (int64_t j = j0; j < j1; ++j) {
    if (flag[j] != 0) idx[o++] = (int)j;
    flag[j] = 0;
  }
  const int K = part[1023];
  if (t < 16 && K + t < (K + 15) / 16 * 16) idx[K + t] = 0;
  if (t == 0) *count = K;
}

// Bu[q][u] = B64[q][idx[u]] for u < K = *kdev, 0 up to K rounded up to 16.
__global__ __launch_bounds__(256) void k_cert_compact(const double* B64, int64_t ld, const int* idx,
                                                      const int* kdev, int nq, double* Bu) {
  const int q = blockIdx.y;
  const int K = *kdev;
  const int Kp = (K + 15) / 16 * 16;
  for (int u = blockIdx.x * 256 + threadIdx.x; u < Kp; u += gridDim.x * 256)
    Bu[(int64_t)q * ld + u] = u < K ? B64[(int64_t)q * ld + idx[u]] : 0.0;
}

// From U64 = X beta (FP64): the loss f, F*(-zeta) with zeta = -grad f(u) (partials per chunk),
// R64 = grad f(u), and the slot's new base (e_0 = u - y or u_0 and r_0).
__global__ __launch_bounds__(256) void k_cert_resid(MixedDev md, const int* list, int nq,
                                                    const double* U64, double* R64,
                                                    double* part, int nchunk, int64_t chunk) {
  __shared__ double red[8];
  const int q = blockIdx.y;
  if (q >= nq) return;
  const int slot = list[q];
  const MemberDev& mb = md.mem[md.st[slot].member];
  const int loss = mb.loss;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(md.n_pad, i0 + chunk);
  double ls = 0.0, fs = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    double r = 0.0, b0 = 0.0, b1 = 0.0;
    if (i < md.n) {
      const double u = U64[(int64_t)q * md.n_pad + i];
      const double y = mb.y[i];
      if (loss == LOSS_LS) {
        const double e = u - y;
        r = 2.0 * e;
        ls += e * e;
        fs += 0.25 * r * r + y * r;
        b0 = e;
      } else {
        r = loss_grad(loss, u, y);
        ls += loss_val(loss, u, y);
        fs += fstar_term(loss, u, y);
        b0 = u;
        b1 = r;
      }
    }
    R64[(int64_t)q * md.n_pad + i] = r;
    if (loss == LOSS_LS) {
      md.e0f[(int64_t)slot * md.n_pad + i] = (float)b0;
    } else {
      md.base0[(int64_t)slot * md.n_pad + i] = b0;
      md.base1[(int64_t)slot * md.n_pad + i] = b1;
    }
  }
  ls = block_reduce(ls, red, OpAdd(), 0.0);
  fs = block_reduce(fs, red + 4, OpAdd(), 0.0);
  if (threadIdx.x == 0) {
    part[((int64_t)q * nchunk + blockIdx.x) * 2] = ls;
    part[((int64_t)q * nchunk + blockIdx.x) * 2 + 1] = fs;
  }
}

// A re-centre keeps the momentum of Alg. 3 when the slot advanced in the latest cycle: the
// iterate before the certified one is still in the ring, the operand of the next X pass still
// holds bf16(beta^{t+1} - beta_0) against the old base, and the ring of X-products holds
// X~ bf16(beta^t - beta_0). Moving the base point is a change of numerical representation, not a
// restart of the method.
__device__ __forceinline__ bool keeps_momentum(const NodeDev* st, int cyc) {
  return st->need_base == 0 && st->iter > 1 && st->last_ring == cyc % 3;
}

// Per certified slot: P = f + 2 lambda2 g, D = -F* - 2 lambda2 g*(X^T zeta / (2 lambda2)) with
// X^T zeta = -H64 (FP64 weak-duality bound, Sec. 3.4). Keeps the best certified P (and its
// beta) and D; finishes the slot or re-centres it on the certified iterate.
template <int E>
__global__ __launch_bounds__(1024) void k_cert_finish(MixedDev md, const int* list, int nq,
                                                      const double* B64, const double* H64,
                                                      const double* part, int nchunk) {
  __shared__ ProxSmem sm;
  const int q = blockIdx.x;
  if (q >= nq) return;
  const int slot = list[q];
  NodeDev* st = md.st + slot;
  const int64_t p = md.p;
  const int cyc = *md.cycle + 1;  // the cycle the slot runs next (the counter holds the last one)
  const bool keep = keeps_momentum(st, cyc);
  const uint8_t* cl = md.cls + (int64_t)slot * md.ldp;
  __shared__ double vbuf[ProxVals<E>::nl * kProxThreads];
  ProxVals<E> hv;
  hv.sl = vbuf;
  uint64_t cb = 0;
  // eigen-perspective shift s: the gradient at beta is X^T grad f(X beta) - 2 s beta, the
  // objective loses s ||beta||^2 and the bound gains it (App. D.2); 0 for the perspective bound
  const MemberDev& mb = md.mem[st->member];
  const double shift = mb.shift;
  const double two_le = 2.0 * (mb.lam2 + shift);
  double bsq = 0.0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
    if (j < p) {
      const double b = B64[(int64_t)q * md.ldp + j];
      hv.set(s, fabs(H64[(int64_t)q * md.ldp + j] - 2.0 * shift * b));
      bsq += b * b;
      cb |= (uint64_t)cl[j] << (2 * s);
    } else {
      hv.set(s, 0.0);
      cb |= (uint64_t)CLS_PAD << (2 * s);
    }
  }
  const double gs = gstar_node<E>([&](int s) { return hv.get(s); }, two_le, cb, st->kp,
                                  st->nfree, mb.M, sm);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nchunk; i += blockDim.x) {
    acc[0] += part[((int64_t)q * nchunk + i) * 2];
    acc[1] += part[((int64_t)q * nchunk + i) * 2 + 1];
  }
  acc[2] = bsq;
  block_sum_n<3>(acc, sm);
  if (threadIdx.x == 0) {
    const double sq = shift != 0.0 ? acc[2] : 0.0;
    const double P = acc[0] - shift * sq + two_le * st->g_new;  // g of the gathered iterate
    const double D = -acc[1] + shift * sq - two_le * gs;
    int improve = 0;
    if (P < st->P_cert) { st->P_cert = P; improve = 1; }
    if (D > st->D_cert) { st->D_cert = D; improve |= 2; }
    st->b_int0 = improve;
    const double gap = (st->P_cert - st->D_cert) / fmax(fabs(st->P_cert), 1.0);
    int status = kRunning;
    if (!(P == P) || !(D == D)) status = 3;
    else if (gap <= st->tol) status = 0;
    else if (isfinite(st->incumbent) && st->D_cert > st->incumbent) status = 5;
    else if (st->iter >= st->max_iter) status = 1;
    else if (isfinite(st->incumbent) && st->P_cert < st->incumbent) status = 6;
    if (status != kRunning) {
      st->status = status;
      st->done = 1;
    } else {
      // re-centre on this iterate
      st->recentres += 1;
      if (keep) {
        st->rebase = 1;
      } else {  // no previous iterate: start the momentum afresh (phi = 1)
        st->primed = 0;
        st->phi = 1.0;
        st->c = 0.25;
        st->L_prev = HUGE_VAL;
      }
      st->P_best = P;
      st->D_best = D;
      st->mgap_ref = HUGE_VAL;
      st->since_improve = 0;
      st->since_recentre = 0;
    }
    st->want_cert = 0;
    st->need_base = 0;
  }
  __syncthreads();
  const bool improve = (st->b_int0 & 1) != 0;
  const bool improve_d = (st->b_int0 & 2) != 0;
  const bool done = st->done != 0;
  const bool fresh = !done && !keep;  // the ring, the operand and the products start at the base
  for (int64_t j = threadIdx.x; j < md.ldp; j += blockDim.x) {
    const double bj = B64[(int64_t)q * md.ldp + j];
    if (improve) md.bres[(int64_t)slot * md.ldp + j] = bj;
    if (improve_d) md.bdual[(int64_t)slot * md.ldp + j] = bj;
    if (!done) {
      md.beta0[(int64_t)slot * md.ldp + j] = bj;
      md.H0[(int64_t)slot * md.ldp + j] = H64[(int64_t)q * md.ldp + j];
    }
    if (fresh)
      for (int r = 0; r < 3; ++r) md.bring[(int64_t)r * md.bring_stride + (int64_t)slot * md.ldp + j] = bj;
    if (!keep || done) md.dop[frag_index(slot, j, md.S_pad >> 5)] = 0;
  }
  if ((!keep || done) && threadIdx.x == 0) md.sn[slot] = 0;
  if (fresh) {
    for (int64_t i = threadIdx.x; i < md.n_pad; i += blockDim.x) {
      md.dU[(int64_t)slot * md.n_pad + i] = 0.f;
      md.dU[md.dU_ring + (int64_t)slot * md.n_pad + i] = 0.f;
    }
  }
}

// Admission from the cold start beta = 0 (the base quantities are the same for every node of
// a problem: u_0 = 0, r_0 = grad f(0), H_0 = X^T r_0). The slot's state (with its problem) has
// been written before this kernel.
__global__ __launch_bounds__(256) void k_admit(MixedDev md, const int* list, int nq) {
  const int q = blockIdx.y;
  if (q >= nq) return;
  const int slot = list[q];
  const MemberDev& mb = md.mem[md.st[slot].member];
  const double* H0_cold = mb.H0c;
  const double* base0_cold = mb.b0c;
  const double* base1_cold = mb.b1c;
  const int64_t stride = (int64_t)gridDim.x * 256;
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // no selection history for a new node
    md.prevhead[(int64_t)slot * 65] = 0;
    md.prevtop[(int64_t)slot * 65] = 0;
    md.sn[slot] = 0;
  }
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < md.ldp; j += stride) {
    const int64_t o = (int64_t)slot * md.ldp + j;
    for (int r = 0; r < 3; ++r) md.bring[(int64_t)r * md.bring_stride + o] = 0.0;
    md.beta0[o] = 0.0;
    md.bres[o] = 0.0;
    md.bdual[o] = 0.0;
    md.H0[o] = H0_cold[j];
    md.dop[frag_index(slot, j, md.S_pad >> 5)] = 0;
  }
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < md.n_pad; i += stride) {
    const int64_t o = (int64_t)slot * md.n_pad + i;
    if (mb.loss == LOSS_LS) {
      md.e0f[o] = (float)base0_cold[i];
    } else {
      md.base0[o] = base0_cold[i];
      md.base1[o] = base1_cold[i];
    }
    md.dU[o] = 0.f;
    md.dU[md.dU_ring + o] = 0.f;
    md.gop[frag_index(slot, i, md.S_pad >> 5)] = 0;
    md.gop_r[(int64_t)slot * md.n_pad + i] = 0;
  }
}

void launch_admit(const MixedDev& md, const int* list, int nq, hipStream_t s) {
  hipLaunchKernelGGL(k_admit, dim3(16, (unsigned)nq), dim3(256), 0, s, md, list, nq);
}

// dst (nq x p, contiguous) = rows list[q] of src (leading dimension ld).
__global__ __launch_bounds__(256) void k_gather_rows(const double* src, int64_t ld, const int* list,
                                                     int nq, int64_t p, double* dst) {
  const int q = blockIdx.y;
  if (q >= nq) return;
  const double* r = src + (int64_t)list[q] * ld;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p; j += (int64_t)gridDim.x * 256)
    dst[(int64_t)q * p + j] = r[j];
}

void launch_gather_rows(const double* src, int64_t ld, const int* list, int nq, int64_t p,
                        double* dst, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(8, (unsigned)nq), dim3(256), 0, s, src, ld, list, nq, p,
                     dst);
}

// =====================================================================================
// Operand order by support (the X pass reads only the prefix of X~'s permuted columns where some
// slot's operand is nonzero)
// =====================================================================================

__global__ __launch_bounds__(256) void k_perm_flags(MixedDev md, uint8_t* flag) {
  const int slot = blockIdx.y;
  const NodeDev* st = md.st + slot;
  if (!slot_running(st)) return;
  // the three iterates of the ring (the latest and the two before it), the base point, the
  // operand in flight (after a re-centre that kept the momentum it is measured from the previous
  // base point) and its strays
  const double* b = md.bring + (int64_t)slot * md.ldp;
  const double* b0 = md.beta0 + (int64_t)slot * md.ldp;
  const int64_t rs = md.bring_stride;
  const int64_t nbk = md.S_pad >> 5;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < md.p; j += (int64_t)gridDim.x * 256)
    if (b[j] != 0.0 || b[rs + j] != 0.0 || b[2 * rs + j] != 0.0 || b0[j] != 0.0 ||
        (md.dop[frag_index(slot, md.pinv[j], nbk)] & 0x7fffu) != 0)
      flag[j] = 1;
  if (blockIdx.x == 0 && (int)threadIdx.x < md.sn[slot])
    flag[md.sj[(int64_t)slot * kStrayCap + threadIdx.x]] = 1;
}

void launch_perm_flags(const MixedDev& md, uint8_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_flags, dim3(4, (unsigned)md.slots), dim3(256), 0, s, md, flag);
}

__global__ __launch_bounds__(1024) void k_perm_build(uint8_t* flag, int64_t p, int64_t ldp,
                                                     int* perm, int* pinv, int* count) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int64_t per = (p + 1023) / 1024;
  const int64_t j0 = min((int64_t)t * per, p), j1 = min(j0 + per, p);
  int c = 0;
  for (int64_t j = j0; j < j1; ++j) c += flag[j] != 0;
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan of the flagged counts
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  const int U = part[1023];
  int f = part[t] - c;                    // flagged coordinates before j0
  int u = U + (int)(j0 - f);              // unflagged coordinates go after all flagged ones
  for (int64_t j = j0; j < j1; ++j) {
    const int pos = flag[j] != 0 ? f++ : u++;
    pinv[j] = pos;
    perm[pos] = (int)j;
    flag[j] = 0;
  }
  for (int64_t j = p + t; j < ldp; j += 1024) {
    pinv[j] = (int)j;
    perm[j] = (int)j;
  }
  if (t == 0) *count = U;
}

void launch_perm_build(uint8_t* flag, int64_t p, int64_t ldp, int* perm, int* pinv, int* count,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_perm_build, dim3(1), dim3(1024), 0, s, flag, p, ldp, perm, pinv, count);
}

__global__ __launch_bounds__(256) void k_perm_operand(MixedDev md, const uint16_t* dop_old,
                                                      const int* pinv_old, const int* pinv_new) {
  const int slot = blockIdx.y;
  // a slot that does not run keeps its operand where it is: it is zero (done, parked, free) or,
  // for a slot at its iteration cap, never read again
  if (!slot_running(md.st + slot)) return;
  const int64_t nbk = md.S_pad >> 5;
  int ext = 0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < md.p; j += (int64_t)gridDim.x * 256) {
    const uint16_t d = dop_old[frag_index(slot, pinv_old[j], nbk)];
    const int pos = pinv_new[j];
    md.dop[frag_index(slot, pos, nbk)] = d;
    if ((d & 0x7fffu) != 0) ext = max(ext, pos + 1);
  }
  ext = wave_max(ext);
  if ((threadIdx.x & 63) == 0 && ext > 0) {
    atomicMax(md.keff, ext);
    atomicMax(md.keff + 1, ext);
  }
}

void launch_perm_operand(const MixedDev& md, const uint16_t* dop_old, const int* pinv_old,
                         const int* pinv_new, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_operand, dim3(8, (unsigned)md.slots), dim3(256), 0, s, md, dop_old,
                     pinv_old, pinv_new);
}

// 64 positions x 64 rows per block through LDS, 16-byte global accesses: thread t reads 8
// consecutive rows i of design row perm[u] (u = t / 8 + 32 h) and scatters them into the
// transposed tile; it then writes 8 consecutive positions of one row of Xb per store.
__global__ __launch_bounds__(256) void k_perm_design(const uint16_t* __restrict__ Xbt,
                                                     int64_t n_pad, const int* __restrict__ perm,
                                                     int64_t p, uint16_t* __restrict__ Xb,
                                                     int64_t ldp) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  __shared__ __attribute__((aligned(16))) uint16_t tile[64][72];  // [i][u]
  const int64_t u0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  const int t = threadIdx.x;
  const int c8 = (t & 7) * 8;  // 8 rows i (load) or 8 positions u (store)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = (t >> 3) + 32 * h;  // position within the tile
    const int64_t u = u0 + r;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (u < p) v = *reinterpret_cast<const u32x4*>(Xbt + (int64_t)perm[u] * n_pad + i0 + c8);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      tile[c8 + 2 * e][r] = (uint16_t)(v[e] & 0xffffu);
      tile[c8 + 2 * e + 1][r] = (uint16_t)(v[e] >> 16);
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = (t >> 3) + 32 * h;
    const int64_t u = u0 + c8;
    const u32x4 v = *reinterpret_cast<const u32x4*>(&tile[i][c8]);
    if (u + 8 <= p) {
      *reinterpret_cast<u32x4*>(Xb + (i0 + i) * ldp + u) = v;
    } else {
      for (int e = 0; e < 8 && u + e < p; ++e)
        Xb[(i0 + i) * ldp + u + e] = (uint16_t)((v[e >> 1] >> (16 * (e & 1))) & 0xffffu);
    }
  }
}

void launch_perm_design(const uint16_t* Xbt, int64_t n_pad, const int* perm, int64_t p,
                        uint16_t* Xb, int64_t ldp, hipStream_t s) {
  const dim3 grid((unsigned)((p + 63) / 64), (unsigned)(n_pad / 64));
  hipLaunchKernelGGL(k_perm_design, grid, dim3(256), 0, s, Xbt, n_pad, perm, p, Xb, ldp);
}

// dst[r][c] = src[r][c] widened to FP64, r < rows, c < cols (leading dimensions ld, ldd).
template <typename XT>
__global__ __launch_bounds__(256) void k_widen(const XT* __restrict__ src, int64_t ld, int64_t rows,
                                               int64_t cols, double* __restrict__ dst, int64_t ldd) {
  const int64_t r = blockIdx.y;
  if (r >= rows) return;
  const XT* a = src + r * ld;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < cols; c += (int64_t)gridDim.x * 256)
    dst[r * ldd + c] = XLoad<XT>::get(a, (size_t)c);
}

void launch_widen(int xtype, const void* src, int64_t ld, int64_t rows, int64_t cols, double* dst,
                  int64_t ldd, hipStream_t s) {
  if (rows <= 0) return;
  const dim3 grid((unsigned)std::min<int64_t>((cols + 255) / 256, 32), (unsigned)rows);
  if (xtype == XT_F64)
    hipLaunchKernelGGL(k_widen<double>, grid, dim3(256), 0, s, (const double*)src, ld, rows, cols, dst, ldd);
  else if (xtype == XT_F32)
    hipLaunchKernelGGL(k_widen<float>, grid, dim3(256), 0, s, (const float*)src, ld, rows, cols, dst, ldd);
  else
    hipLaunchKernelGGL(k_widen<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)src, ld, rows, cols, dst, ldd);
}

// Least squares: X^T grad f(X beta) = 2 X^T X beta - 2 X^T y. H[q][j] holds (X^T X beta_q)_j on
// entry and the gradient on exit; h0 = X^T grad f(0) = -2 X^T y of slot list[q]'s problem.
__global__ __launch_bounds__(256) void k_gram_finish(double* H, int64_t ld, int64_t p,
                                                     MixedDev md, const int* list) {
  const int q = blockIdx.y;
  const double* h0 = md.mem[md.st[list[q]].member].H0c;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p; j += (int64_t)gridDim.x * 256)
    H[(int64_t)q * ld + j] = 2.0 * H[(int64_t)q * ld + j] + h0[j];
}

void launch_gram_finish(double* H, int64_t ld, int64_t p, int nq, const MixedDev& md,
                        const int* list, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_gram_finish, dim3(8, (unsigned)nq), dim3(256), 0, s, H, ld, p, md, list);
}

// Zero a slot's operand rows (retired or empty slots must not contribute to the products).
__global__ __launch_bounds__(256) void k_slot_clear(MixedDev md, int slot) {
  if (blockIdx.x == 0 && threadIdx.x == 0) md.sn[slot] = 0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < md.ldp; j += (int64_t)gridDim.x * 256)
    md.dop[frag_index(slot, j, md.S_pad >> 5)] = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < md.n_pad; i += (int64_t)gridDim.x * 256) {
    md.gop[frag_index(slot, i, md.S_pad >> 5)] = 0;
    md.gop_r[(int64_t)slot * md.n_pad + i] = 0;
    md.dU[(int64_t)slot * md.n_pad + i] = 0.f;
    md.dU[md.dU_ring + (int64_t)slot * md.n_pad + i] = 0.f;
  }
}

// X~ (n_pad x ldp) and X~^T (ldp x n_pad) in BF16 from X in its stored precision.
template <typename XT>
__global__ __launch_bounds__(256) void k_make_bf16(const XT* __restrict__ X, int64_t ldx,
                                                   int64_t n, int64_t p, int64_t n_pad,
                                                   int64_t ldp, uint16_t* __restrict__ Xb,
                                                   uint16_t* __restrict__ Xbt) {
  __shared__ uint16_t tile[32][33];
  const int64_t j0 = (int64_t)blockIdx.x * 32, i0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, j = j0 + tx;
    uint16_t v = 0;
    if (i < n && j < p) v = float_to_bf16((float)XLoad<XT>::get(X, (size_t)(i * ldx + j)));
    if (i < n_pad && j < ldp) Xb[i * ldp + j] = v;
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + r, i = i0 + tx;
    if (j < ldp && i < n_pad) Xbt[j * n_pad + i] = tile[tx][r];
  }
}

// ------------------------------------------------------------------ launchers

void launch_make_bf16(int xtype, const void* X, int64_t ldx, int64_t n, int64_t p, int64_t n_pad,
                      int64_t ldp, uint16_t* Xb, uint16_t* Xbt, hipStream_t s) {
  dim3 grid((unsigned)((ldp + 31) / 32), (unsigned)((n_pad + 31) / 32));
  if (xtype == XT_F64)
    hipLaunchKernelGGL(k_make_bf16<double>, grid, dim3(256), 0, s, (const double*)X, ldx, n, p, n_pad, ldp, Xb, Xbt);
  else if (xtype == XT_F32)
    hipLaunchKernelGGL(k_make_bf16<float>, grid, dim3(256), 0, s, (const float*)X, ldx, n, p, n_pad, ldp, Xb, Xbt);
  else
    hipLaunchKernelGGL(k_make_bf16<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)X, ldx, n, p, n_pad, ldp, Xb, Xbt);
}

// One product launch in the row tiling rt (8: 256 rows, 4: 128 rows, 2: 64 rows per
// workgroup); with e0, the launch itself records its start and end (no separate event packets).
template <int PASS>
static void launch_bf16(int rt, dim3 grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                        const GemmArgs& g, int mt, int ks, int per, int* bump, int* extent) {
  if (rt == 2) {
    if (e0 != nullptr)
      hipExtLaunchKernelGGL((k_gemm_bf16<PASS, 2>), grid, dim3(256), 0, s, e0, e1, 0, g, mt, ks,
                            per, bump, extent);
    else
      hipLaunchKernelGGL((k_gemm_bf16<PASS, 2>), grid, dim3(256), 0, s, g, mt, ks, per, bump,
                         extent);
  } else if (rt == 4) {
    if (e0 != nullptr)
      hipExtLaunchKernelGGL((k_gemm_bf16<PASS, 4>), grid, dim3(256), 0, s, e0, e1, 0, g, mt, ks,
                            per, bump, extent);
    else
      hipLaunchKernelGGL((k_gemm_bf16<PASS, 4>), grid, dim3(256), 0, s, g, mt, ks, per, bump,
                         extent);
  } else {
    if (e0 != nullptr)
      hipExtLaunchKernelGGL((k_gemm_bf16<PASS, 8>), grid, dim3(256), 0, s, e0, e1, 0, g, mt, ks,
                            per, bump, extent);
    else
      hipLaunchKernelGGL((k_gemm_bf16<PASS, 8>), grid, dim3(256), 0, s, g, mt, ks, per, bump,
                         extent);
  }
}

void launch_gemm_x(const MixedDev& md, hipStream_t s, bool advance, hipEvent_t e0, hipEvent_t e1) {
  GemmArgs g;
  g.A = md.Xb;
  g.lda = md.ldp;
  g.B = md.dop;
  g.nb = md.S_pad / 32;
  g.M = md.n_pad;
  g.K = md.ldp;
  g.kchunk = md.x_kchunk;
  g.C = md.dUp;
  g.ldc = md.n_pad;
  g.c_split_stride = md.dUp_split;
  const int mt = (int)(md.n_pad / (32 * md.x_rt)), per = (mt * md.ksx + 7) / 8;
  dim3 grid((unsigned)(8 * per), (unsigned)(md.S_pad / GT_N));
  int* bump = advance ? md.cycle : nullptr;
  launch_bf16<0>(md.x_rt, grid, s, e0, e1, g, mt, md.ksx, per, bump, md.keff);
}

void launch_gemm_xt(const MixedDev& md, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  GemmArgs g;
  g.A = md.Xbt;
  g.lda = md.n_pad;
  g.B = md.gop;
  g.nb = md.S_pad / 32;
  g.M = md.ldp;
  g.K = md.n_pad;
  g.kchunk = md.xt_kchunk;
  g.C = md.dH;
  g.ldc = md.ldp;
  g.c_split_stride = md.dH_split;
  const int mt = (int)(md.ldp / (32 * md.xt_rt)), per = (mt * md.ksplit + 7) / 8;
  dim3 grid((unsigned)(8 * per), (unsigned)(md.S_pad / GT_N));
  launch_bf16<1>(md.xt_rt, grid, s, e0, e1, g, mt, md.ksplit, per, nullptr, nullptr);
}

void launch_mixed_loss(const MixedDev& md, hipStream_t s) {
  const dim3 grid((unsigned)md.nrt, (unsigned)md.slots);
  if (md.loss_kinds & 1) hipLaunchKernelGGL(k_mixed_loss<true>, grid, dim3(256), 0, s, md);
  if (md.loss_kinds & 2) hipLaunchKernelGGL(k_mixed_loss<false>, grid, dim3(256), 0, s, md);
}

void launch_mixed_decide(const MixedDev& md, hipStream_t s) {
  hipLaunchKernelGGL(k_mixed_decide, dim3(kDecideBlocks, (unsigned)md.slots), dim3(256), 0, s, md);
}

#define CGL_E_SWITCH(E_, CALL)   \
  switch (E_) {                  \
    case 1: { constexpr int EE = 1; CALL; break; }   \
    case 2: { constexpr int EE = 2; CALL; break; }   \
    case 4: { constexpr int EE = 4; CALL; break; }   \
    case 6: { constexpr int EE = 6; CALL; break; }   \
    case 8: { constexpr int EE = 8; CALL; break; }   \
    case 10: { constexpr int EE = 10; CALL; break; } \
    case 12: { constexpr int EE = 12; CALL; break; } \
    case 16: { constexpr int EE = 16; CALL; break; } \
    case 20: { constexpr int EE = 20; CALL; break; } \
    case 24: { constexpr int EE = 24; CALL; break; } \
    case 32: { constexpr int EE = 32; CALL; break; } \
    default: break;              \
  }

void launch_mixed_node(const MixedDev& md, hipStream_t s) {
  const int E = prox_elems(md.p);
  CGL_E_SWITCH(E, hipLaunchKernelGGL(k_mixed_node<EE>, dim3(md.slots), dim3(kProxThreads), 0, s, md));
}

void launch_transpose(int xtype, const void* X, int64_t ldx, int64_t n, int64_t p, int64_t n_pad,
                      void* Xt, hipStream_t s) {
  dim3 grid((unsigned)((p + 31) / 32), (unsigned)((n_pad + 31) / 32));
  if (xtype == XT_F64)
    hipLaunchKernelGGL(k_transpose<double>, grid, dim3(256), 0, s, (const double*)X, ldx, n, p, n_pad, (double*)Xt);
  else if (xtype == XT_F32)
    hipLaunchKernelGGL(k_transpose<float>, grid, dim3(256), 0, s, (const float*)X, ldx, n, p, n_pad, (float*)Xt);
  else
    hipLaunchKernelGGL(k_transpose<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)X, ldx, n, p, n_pad, (uint16_t*)Xt);
}

// Launch shape of the FP64 products: node tile 32 when that pads Q no further than 16 would, else
// 16; split K until there are about 4 workgroups per compute unit, each chunk >= 32 steps of 16
// and the partials within part_cap bytes.
struct F64Launch {
  int nt;
  int64_t mblocks, qblocks, ks, chunk;
};
static F64Launch f64_launch(int64_t M, int64_t K, int Q, size_t part_cap) {
  F64Launch l;
  l.nt = ((Q + 31) / 32 * 32 == (Q + 15) / 16 * 16) ? 2 : 1;
  l.mblocks = (M + 64 * F64_RT - 1) / (64 * F64_RT);
  l.qblocks = (Q + 16 * l.nt - 1) / (16 * l.nt);
  const int64_t steps = std::max<int64_t>(1, (K + 15) / 16);
  int64_t ks = (1024 + l.mblocks * l.qblocks - 1) / (l.mblocks * l.qblocks);
  ks = std::min<int64_t>(ks, std::max<int64_t>(1, steps / 32));
  ks = std::min<int64_t>(ks, (int64_t)(part_cap / ((size_t)Q * M * sizeof(double))));
  ks = std::max<int64_t>(ks, 1);
  l.chunk = (steps + ks - 1) / ks * 16;
  l.ks = std::max<int64_t>(1, (K + l.chunk - 1) / l.chunk);
  return l;
}

static void launch_f64_reduce(const double* part, int64_t ks, int Q, int64_t M, double* C,
                              int64_t ldc, hipStream_t s) {
  dim3 rg((unsigned)std::min<int64_t>((M + 255) / 256, 64), (unsigned)Q);
  hipLaunchKernelGGL(k_gemm_f64_reduce, rg, dim3(256), 0, s, part, (int)ks, Q, M, C, ldc);
}

void launch_gemm_f64(int xtype, const void* A, int64_t lda, int64_t M, int64_t K,
                     const double* B, int64_t ldb, int Q, double* C, int64_t ldc, double* part,
                     size_t part_cap, hipStream_t s) {
  if (Q <= 0 || M <= 0) return;
  const F64Launch l = f64_launch(M, K, Q, part_cap);
  F64GemmArgs g{A, lda, B, ldb, M, K, Q, l.chunk, l.ks > 1 ? part : C, l.ks > 1 ? M : ldc};
  dim3 grid((unsigned)l.mblocks, (unsigned)l.qblocks, (unsigned)l.ks);
#define CGL_F64_CALL(T)                                                              \
  if (l.nt == 2) hipLaunchKernelGGL((k_gemm_f64<T, 2>), grid, dim3(256), 0, s, g); \
  else hipLaunchKernelGGL((k_gemm_f64<T, 1>), grid, dim3(256), 0, s, g);
  if (xtype == XT_F64) { CGL_F64_CALL(double) }
  else if (xtype == XT_F32) { CGL_F64_CALL(float) }
  else { CGL_F64_CALL(uint16_t) }
#undef CGL_F64_CALL
  if (l.ks > 1) launch_f64_reduce(part, l.ks, Q, M, C, ldc, s);
}

void launch_gemm_f64_rows(int xtype, const void* At, int64_t ldat, const int* idx, int64_t M,
                          int64_t K, const int* kdev, const double* B, int64_t ldb, int Q,
                          double* C, int64_t ldc, double* part, size_t part_cap, hipStream_t s) {
  if (Q <= 0 || M <= 0) return;
  const F64Launch l = f64_launch(M, K, Q, part_cap);
  F64RowsArgs g{At, ldat, idx, B, ldb, M, K, Q, l.chunk, l.ks > 1 ? part : C, l.ks > 1 ? M : ldc,
                kdev};
  dim3 grid((unsigned)l.mblocks, (unsigned)l.qblocks, (unsigned)l.ks);
#define CGL_F64_CALL(T)                                                                   \
  if (l.nt == 2) hipLaunchKernelGGL((k_gemm_f64_rows<T, 2>), grid, dim3(256), 0, s, g); \
  else hipLaunchKernelGGL((k_gemm_f64_rows<T, 1>), grid, dim3(256), 0, s, g);
  if (xtype == XT_F64) { CGL_F64_CALL(double) }
  else if (xtype == XT_F32) { CGL_F64_CALL(float) }
  else { CGL_F64_CALL(uint16_t) }
#undef CGL_F64_CALL
  if (l.ks > 1) launch_f64_reduce(part, l.ks, Q, M, C, ldc, s);
}

void launch_cert_gather(const MixedDev& md, const int* list, int nq, double* B64, uint8_t* flag,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_cert_gather, dim3(8, (unsigned)nq), dim3(256), 0, s, md, list, nq, B64,
                     flag);
}

void launch_cert_support(uint8_t* flag, int64_t p, int* idx, int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_cert_support, dim3(1), dim3(1024), 0, s, flag, p, idx, count);
}

void launch_cert_compact(const double* B64, int64_t ld, const int* idx, const int* kdev,
                         int64_t Kmax, int nq, double* Bu, hipStream_t s) {
  if (nq <= 0) return;
  const int64_t Kp = (Kmax + 15) / 16 * 16;
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((Kp + 255) / 256, 16));
  hipLaunchKernelGGL(k_cert_compact, dim3(gx, (unsigned)nq), dim3(256), 0, s, B64, ld, idx, kdev,
                     nq, Bu);
}

void launch_cert_resid(const MixedDev& md, const int* list, int nq, const double* U64,
                       double* R64, double* part, int nchunk, int64_t chunk, hipStream_t s) {
  hipLaunchKernelGGL(k_cert_resid, dim3((unsigned)nchunk, (unsigned)nq), dim3(256), 0, s, md,
                     list, nq, U64, R64, part, nchunk, chunk);
}

void launch_cert_finish(const MixedDev& md, const int* list, int nq, const double* B64,
                        const double* H64, const double* part, int nchunk, hipStream_t s) {
  const int E = prox_elems(md.p);
  CGL_E_SWITCH(E, hipLaunchKernelGGL(k_cert_finish<EE>, dim3((unsigned)nq), dim3(kProxThreads), 0, s, md, list, nq, B64, H64, part, nchunk));
}

void launch_slot_clear(const MixedDev& md, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_slot_clear, dim3(16), dim3(256), 0, s, md, slot);
}

}  // namespace cgl

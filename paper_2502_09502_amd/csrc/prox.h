// Exact node prox of g (Alg. 1 through the Moreau identity, Sec. 3.2-3.3), g (Alg. 2) and the
// TopSum-of-Huber conjugate (Lemma 2) for one node per 1024-thread workgroup.
//
// Structure used (derived from Lemma 3 and Alg. 1). With u = rho |w_F| sorted decreasingly, the
// initial values of Alg. 1 are huber_prox(rho, u_j) on the k' head positions and u_j on the tail;
// both runs are already non-increasing, so the only isotonic violation is at the head/tail
// junction and pooling produces at most one block [a, b] with a <= k' < b. Its value v* is the
// root of the increasing, piecewise-linear function
//
//   phi(v) = sum_{head} [ (v - u_j) + rho min(v, M) ]_+  -  sum_{tail} (u_j - v)_+ ,
//
// (the stationarity of the pooled block objective: head members are those with
// huber_prox(rho, u_j) < v, tail members those with u_j > v). Every pooled value equals v*: the
// isotonic solution is nu_j = max(huber_prox(rho, u_j), v*) on the head and min(u_j, v*) on the
// tail, so after the Moreau identity (|beta_j| = (u_j - nu_j) / rho)
//
//   |beta_j| = ( u_j - max(c_j, v*) )_+ / rho,   c_j = huber_prox(rho, u_j) on the head,
//                                                c_j = 0 on the tail,
//
// i.e. ridge-and-clip min(rho|w_j|/(1+rho), M) for head non-members, soft threshold
// |w_j| - v*/rho for block members and 0 for the rest of the tail; signs follow w.
//
// GPU realisation, no sort of the p entries:
//  * head: the k'+1 largest u (ties: smaller index first) by k'+1 rounds of wave-wide argmax in
//    each of the 16 waves, merged by one wave; the result comes out sorted (byte-wise radix
//    select on the FP64 bit patterns for k' > 63);
//  * v*: a monotone fixed-point iteration. From a lower bound v_0 (the previous iteration's v*
//    when phi(v_0) <= 0, else 0), take the tail set A = {u > v_k} (one block reduction of its
//    count and sum) and let v_{k+1} be the exact root of H(v) - sum_A (u - v), solved in closed
//    form over the <= k'+1 head breakpoints. That function lies above phi on [v_k, inf), so
//    v_k <= v_{k+1} <= v*; when A stops shrinking, phi(v_{k+1}) = 0 exactly. All sums are FP64.
#pragma once

#include <limits.h>

#include "common.h"

namespace cgl {

constexpr int kProxThreads = 1024;
constexpr int kProxWaves = kProxThreads / kWave;
constexpr int kMaxHead = 256;  // supports k' <= 256
constexpr int kWaveSel = 64;   // wave selection handles up to 64 winners (k' <= 63)

enum : uint8_t { CLS_FREE = 0, CLS_ZERO = 1, CLS_ONE = 2, CLS_PAD = 3 };

struct ProxSmem {
  uint32_t cnt[256];                     // radix histogram (k' > 63)
  double cand_v[kProxWaves * kWaveSel];  // per-wave winners
  int cand_i[kProxWaves * kWaveSel];
  double hu[kMaxHead + 1];  // sorted head u values; hu[k'] = largest tail value
  int hidx[kMaxHead + 1];
  double tmp[kMaxHead];
  double redd[kProxWaves * 4];
  uint64_t redu[kProxWaves];
  int redi[kProxWaves];
  int head_fill;
  int ties_left;
  int b_int[4];
  double b_dbl[4];
};

__device__ __forceinline__ uint64_t dbits(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(uint64_t k) { return __longlong_as_double((long long)k); }

__device__ __forceinline__ double bsum(double v, ProxSmem& sm) {
  return block_reduce(v, sm.redd, OpAdd(), 0.0);
}
__device__ __forceinline__ int bsum_i(int v, ProxSmem& sm) {
  return block_reduce(v, sm.redi, OpAdd(), 0);
}
__device__ __forceinline__ double bmax(double v, ProxSmem& sm) {
  return block_reduce(v, sm.redd, OpMax(), -HUGE_VAL);
}
__device__ __forceinline__ uint64_t bor(uint64_t v, ProxSmem& sm) {
  return block_reduce(v, sm.redu, OpOr(), (uint64_t)0);
}
__device__ __forceinline__ uint64_t band(uint64_t v, ProxSmem& sm) {
  return block_reduce(v, sm.redu, OpAnd(), ~(uint64_t)0);
}

// Sum of N values over the block in one pass (N <= 4); every thread receives the totals.
template <int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], ProxSmem& sm) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) sm.redd[i * kProxWaves + wid] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double r = 0.0;
    for (int w = 0; w < kProxWaves; ++w) r += sm.redd[i * kProxWaves + w];
    v[i] = r;
  }
}

// Inclusive suffix scan across the 64 lanes of a wave (lane i gets sum over lanes >= i).
template <typename T>
__device__ __forceinline__ T wave_suffix_incl(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T o = __shfl_down(v, off, kWave);
    if (lane + off < 64) v += o;
  }
  return v;
}

// Wave-wide argmax of (value, index): larger value wins, ties go to the smaller index. Every
// lane receives the winner.
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, kWave);
    const int oi = __shfl_xor(i, off, kWave);
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
  }
}

// The K largest active keys (K <= kWaveSel, K <= number of active keys), sorted decreasingly
// (ties: smaller index first), into sm.hu[0..K) / sm.hidx[0..K). Element s of thread t has index
// s * kProxThreads + t.
template <int E>
__device__ void block_topk(const double (&key)[E], const bool (&act)[E], int K, ProxSmem& sm) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  uint32_t taken = 0;
  for (int r = 0; r < K; ++r) {
    double bv = -1.0;  // keys are >= 0
    int bi = INT_MAX;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int j = s * kProxThreads + (int)threadIdx.x;
      if (act[s] && !((taken >> s) & 1u) && (key[s] > bv || (key[s] == bv && j < bi))) {
        bv = key[s];
        bi = j;
      }
    }
    wave_argmax(bv, bi);
    if (bi != INT_MAX && (bi & (kProxThreads - 1)) == (int)threadIdx.x)
      taken |= 1u << (bi / kProxThreads);
    if (lane == 0) {
      sm.cand_v[wid * kWaveSel + r] = bv;
      sm.cand_i[wid * kWaveSel + r] = bi;
    }
  }
  __syncthreads();
  if (wid == 0) {
    // lane l holds the candidates of waves l / 4 ... : slot q covers wave (q * 4 + l / 16)
    // simpler: candidate c = q * 64 + lane over the flattened list of kProxWaves * K entries
    const int total = kProxWaves * K;
    double cv[kProxWaves];
    int ci[kProxWaves];
#pragma unroll
    for (int q = 0; q < kProxWaves; ++q) {
      const int c = q * 64 + lane;
      if (c < total) {
        const int w = c / K, r = c % K;
        cv[q] = sm.cand_v[w * kWaveSel + r];
        ci[q] = sm.cand_i[w * kWaveSel + r];
      } else {
        cv[q] = -1.0;
        ci[q] = INT_MAX;
      }
    }
    uint32_t tk = 0;
    for (int r = 0; r < K; ++r) {
      double bv = -1.0;
      int bi = INT_MAX, bq = -1;
#pragma unroll
      for (int q = 0; q < kProxWaves; ++q) {
        if (!((tk >> q) & 1u) && (cv[q] > bv || (cv[q] == bv && ci[q] < bi))) {
          bv = cv[q];
          bi = ci[q];
          bq = q;
        }
      }
      double wv = bv;
      int wi = bi;
      wave_argmax(wv, wi);
      if (bq >= 0 && bi == wi && wi != INT_MAX) tk |= 1u << bq;
      if (lane == 0) {
        sm.hu[r] = wv;
        sm.hidx[r] = wi;
      }
    }
  }
  __syncthreads();
}

// Result of a descending radix selection: selected = key > lo, plus `take` of the keys == lo
// when `exact`; when !exact, selected = key >= lo (and the count is exactly the requested one).
struct Select {
  uint64_t lo;
  bool exact;
  int take;
};

// need-th largest among active keys (1 <= need <= number of active keys). Byte-wise radix.
template <int E>
__device__ Select radix_select_desc(const uint64_t (&key)[E], const bool (&act)[E], int need,
                                    ProxSmem& sm) {
  uint64_t o = 0, a = ~(uint64_t)0;
#pragma unroll
  for (int s = 0; s < E; ++s)
    if (act[s]) { o |= key[s]; a &= key[s]; }
  o = bor(o, sm);
  a = band(a, sm);
  const uint64_t diff = o ^ a;
  if (diff == 0) return Select{a, true, need};
  const int hb = 63 - __clzll(diff);
  int shift = (hb >> 3) << 3;
  uint64_t prefix = (shift + 8 >= 64) ? 0 : (a & ~((((uint64_t)1) << (shift + 8)) - 1));
  int remaining = need;
  const int lane = threadIdx.x & 63;
  for (;;) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) sm.cnt[i] = 0;
    __syncthreads();
    const int hs = shift + 8;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      if (act[s] && (hs >= 64 || (key[s] >> hs) == (prefix >> hs)))
        atomicAdd(&sm.cnt[(key[s] >> shift) & 255], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      int c[4];
      int loc = 0;
#pragma unroll
      for (int i = 3; i >= 0; --i) { c[i] = (int)sm.cnt[lane * 4 + i]; loc += c[i]; }
      const int suf = wave_suffix_incl(loc);
      int best = -1, above = 0, binc = 0;
      int run = suf - loc;  // bins of higher lanes
#pragma unroll
      for (int i = 3; i >= 0; --i) {
        const int incl = run + c[i];
        if (best < 0 && incl >= remaining) { best = lane * 4 + i; above = run; binc = c[i]; }
        run = incl;
      }
      int cand = best;  // highest bin whose suffix count reaches `remaining`
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) cand = max(cand, __shfl_xor(cand, off, kWave));
      if (best == cand && best >= 0) {
        sm.b_int[0] = best;
        sm.b_int[1] = above;
        sm.b_int[2] = binc;
      }
    }
    __syncthreads();
    const int b = sm.b_int[0];
    const int above = sm.b_int[1];
    const int binc = sm.b_int[2];
    __syncthreads();
    remaining -= above;
    prefix |= ((uint64_t)b) << shift;
    if (binc == remaining) return Select{prefix, false, 0};
    if (shift == 0) return Select{prefix, true, remaining};
    shift -= 8;
  }
}

// Rank-sort sm.hu[0..kh) decreasingly (ties keep an arbitrary but consistent order).
__device__ __forceinline__ void sort_head_desc(int kh, ProxSmem& sm) {
  for (int i = threadIdx.x; i < kh; i += blockDim.x) sm.tmp[i] = sm.hu[i];
  __syncthreads();
  for (int i = threadIdx.x; i < kh; i += blockDim.x) {
    const double x = sm.tmp[i];
    int r = 0;
    for (int j = 0; j < kh; ++j) {
      const double y = sm.tmp[j];
      r += (y > x || (y == x && j < i)) ? 1 : 0;
    }
    sm.hu[r] = x;
  }
  __syncthreads();
}

// head part of phi: sum over head values hu[0..kh) of [(v - u) + rho min(v, M)]_+
__device__ __forceinline__ double head_part(const double* hu, int kh, double v, double rho,
                                            double M) {
  double acc = 0.0;
  const double pen = rho * fmin(v, M);
  for (int i = 0; i < kh; ++i) {
    const double t = (v - hu[i]) + pen;
    acc += t > 0.0 ? t : 0.0;
  }
  return acc;
}

// Root of psi(v) = H(v) - (S - m v) on [vlo, inf) (psi increasing, psi(vlo) <= 0). Breakpoints
// of H: huber_prox(rho, hu_i, M) and M. Every wave evaluates it (no barrier needed).
__device__ double psi_root(const double* hu, int kh, double vlo, double m, double S, double rho,
                           double M) {
  const int lane = threadIdx.x & 63;
  double a = vlo, b = HUGE_VAL;
  for (int base = 0; base <= kh; base += 64) {
    const int i = base + lane;
    if (i <= kh) {
      const double pt = (i < kh) ? huber_prox(rho, hu[i], M) : M;
      if (pt > vlo) {
        const double ps = head_part(hu, kh, pt, rho, M) - (S - m * pt);
        if (ps <= 0.0) a = fmax(a, pt);
        else b = fmin(b, pt);
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a = fmax(a, __shfl_xor(a, off, kWave));
    b = fmin(b, __shfl_xor(b, off, kWave));
  }
  // membership of the head and the regime of min(v, M) are constant on (a, b)
  const double mid = isinf(b) ? a + fmax(1.0, fabs(a)) : 0.5 * (a + b);
  double nh = 0.0, sh = 0.0;
  for (int i = 0; i < kh; ++i) {
    if (huber_prox(rho, hu[i], M) < mid) { nh += 1.0; sh += hu[i]; }
  }
  double v;
  if (mid <= M) {
    const double den = m + nh * (1.0 + rho);
    v = den > 0.0 ? (S + sh) / den : a;
  } else {
    const double den = m + nh;
    v = den > 0.0 ? (S + sh - rho * M * nh) / den : a;
  }
  return fmin(fmax(v, a), b);
}

// v* over the tail (see the file comment). hu[0..kh): sorted head values. v0: a hint.
template <int E>
__device__ double tail_root(const double (&u)[E], const bool (&tail)[E], const double* hu,
                           int kh, double v0, double rho, double M, ProxSmem& sm) {
  double v = v0 > 0.0 ? v0 : 0.0;
  double m_prev = -1.0;
  bool checked_start = v == 0.0;
  for (int it = 0; it < 4096; ++it) {
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < E; ++s) {
      if (tail[s] && u[s] > v) { acc[0] += 1.0; acc[1] += u[s]; }
    }
    block_sum_n<2>(acc, sm);
    const double m = acc[0], S = acc[1];
    if (!checked_start) {
      checked_start = true;
      if (head_part(hu, kh, v, rho, M) - (S - m * v) > 0.0) {
        // hint above v*: the members at the hint are a subset of those at any v below it, so
        // the root with this set fixed, searched from 0, is a lower bound on v* (and close to it
        // when the hint is)
        v = psi_root(hu, kh, 0.0, m, S, rho, M);
        continue;
      }
    }
    if (m == m_prev) break;  // the member set did not change: v is the root
    v = psi_root(hu, kh, v, m, S, rho, M);
    m_prev = m;
  }
  return v;
}

// Alg. 2 on the head magnitudes |beta| (sorted decreasingly, kh entries, the top of |beta_F|)
// with total s = sum |beta_F|, budget kp.
__device__ __forceinline__ double alg2_from_sorted(const double* mag, int kh, int kp, double s) {
  double g = 0.0;
  for (int j = 0; j < kp; ++j) {
    const double bj = j < kh ? mag[j] : 0.0;
    const double sbar = s / (double)(kp - j);
    if (sbar >= bj) {
      g += (double)(kp - j) * sbar * sbar;
      break;
    }
    g += bj * bj;
    s -= bj;
  }
  return 0.5 * g;
}

struct ProxOut {
  double gval;   // g_node(beta)
  double vstar;  // pooled value (warm start of the next call)
};

// Node prox in registers. w: element s of this thread is index j = s * kProxThreads + tid.
// cls: CLS_*; kp = k - |Z1| (>= 0); nfree = |F|; vhint: previous v* (0 if none).
template <int E>
__device__ ProxOut node_prox(const double (&w)[E], const uint8_t (&cls)[E], int kp, int nfree,
                             double rho, double M, double vhint, double (&beta)[E],
                             ProxSmem& sm) {
  double u[E];
  bool freeb[E];
  double z1sq = 0.0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    u[s] = rho * fabs(w[s]);
    freeb[s] = cls[s] == CLS_FREE;
    beta[s] = 0.0;
    if (cls[s] == CLS_ONE) {
      double b = rho * w[s] / (1.0 + rho);
      b = fmin(fmax(b, -M), M);
      beta[s] = b;
      z1sq += b * b;
    }
  }
  ProxOut out;
  out.vstar = 0.0;
  if (kp <= 0 || nfree == 0) {  // F pinned to zero (no budget left) or empty
    out.gval = 0.5 * bsum(z1sq, sm);
    return out;
  }
  if (kp >= nfree) {  // every free coordinate can take z = 1: ridge-and-clip, g = 1/2 ||beta||^2
    double sq = z1sq;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      if (freeb[s] && w[s] != 0.0) {
        const double b = copysign(fmin(u[s] / (1.0 + rho), M), w[s]);
        beta[s] = b;
        sq += b * b;
      }
    }
    out.gval = 0.5 * bsum(sq, sm);
    return out;
  }
  // ---- head: the kp largest u over F (sorted into sm.hu), and the largest tail value
  bool head[E];
  double umax_tail;
  if (kp + 1 <= kWaveSel) {
    block_topk<E>(u, freeb, kp + 1, sm);
    const double tv = sm.hu[kp - 1];
    const int ti = sm.hidx[kp - 1];
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int j = s * kProxThreads + (int)threadIdx.x;
      head[s] = freeb[s] && (u[s] > tv || (u[s] == tv && j <= ti));
    }
    umax_tail = sm.hu[kp];
  } else {
    uint64_t key[E];
#pragma unroll
    for (int s = 0; s < E; ++s) key[s] = dbits(u[s]);
    const Select sel = radix_select_desc<E>(key, freeb, kp, sm);
    if (threadIdx.x == 0) { sm.head_fill = 0; sm.ties_left = sel.exact ? sel.take : 0; }
    __syncthreads();
    double tmax = -1.0;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      bool h = false;
      if (freeb[s]) {
        if (!sel.exact) h = key[s] >= sel.lo;
        else if (key[s] > sel.lo) h = true;
        else if (key[s] == sel.lo) h = atomicSub(&sm.ties_left, 1) > 0;
      }
      head[s] = h;
      if (h) sm.hu[atomicAdd(&sm.head_fill, 1)] = u[s];
      else if (freeb[s]) tmax = fmax(tmax, u[s]);
    }
    __syncthreads();
    sort_head_desc(kp, sm);
    umax_tail = bmax(tmax, sm);
  }
  // ---- v*
  bool tail[E];
#pragma unroll
  for (int s = 0; s < E; ++s) tail[s] = freeb[s] && !head[s];
  double vstar;
  if (huber_prox(rho, sm.hu[kp - 1], M) >= umax_tail) {
    vstar = umax_tail;  // no isotonic violation at the junction: no pooled block
  } else {
    vstar = tail_root<E>(u, tail, sm.hu, kp, vhint, rho, M, sm);
  }
  out.vstar = vstar;
  // ---- assemble beta; |beta_F| total and Z1 squares in one reduction
  double acc[2] = {0.0, z1sq};
#pragma unroll
  for (int s = 0; s < E; ++s) {
    if (freeb[s]) {
      const double c = head[s] ? huber_prox(rho, u[s], M) : 0.0;
      const double t = u[s] - fmax(c, vstar);
      const double mag = t > 0.0 ? t / rho : 0.0;
      beta[s] = mag > 0.0 ? copysign(mag, w[s]) : 0.0;
      acc[0] += mag;
    }
  }
  // head magnitudes in sorted order (|beta| is monotone in u)
  for (int i = threadIdx.x; i < kp; i += blockDim.x) {
    const double uh = sm.hu[i];
    const double t = uh - fmax(huber_prox(rho, uh, M), vstar);
    sm.tmp[i] = t > 0.0 ? t / rho : 0.0;
  }
  block_sum_n<2>(acc, sm);
  if (threadIdx.x == 0) sm.b_dbl[3] = alg2_from_sorted(sm.tmp, kp, kp, acc[0]);
  __syncthreads();
  out.gval = 0.5 * acc[1] + sm.b_dbl[3];
  __syncthreads();
  return out;
}

// g_node*(a) = sum_{Z1} H_M(a_j) + TopSum_{kp}(H_M(a_F))  (Lemma 2, separable sum rule).
template <int E>
__device__ double gstar_node(const double (&a)[E], const uint8_t (&cls)[E], int kp, int nfree,
                             double M, ProxSmem& sm) {
  double z1 = 0.0;
  bool freeb[E];
  double mag[E];
#pragma unroll
  for (int s = 0; s < E; ++s) {
    freeb[s] = cls[s] == CLS_FREE;
    mag[s] = fabs(a[s]);
    if (cls[s] == CLS_ONE) z1 += huber(a[s], M);
  }
  double top = 0.0;
  if (kp > 0 && nfree > 0) {
    if (kp >= nfree) {
#pragma unroll
      for (int s = 0; s < E; ++s)
        if (freeb[s]) top += huber(a[s], M);
    } else if (kp <= kWaveSel) {
      block_topk<E>(mag, freeb, kp, sm);
      if (threadIdx.x == 0)
        for (int r = 0; r < kp; ++r) top += huber(sm.hu[r], M);
    } else {
      uint64_t key[E];
#pragma unroll
      for (int s = 0; s < E; ++s) key[s] = dbits(mag[s]);
      const Select sel = radix_select_desc<E>(key, freeb, kp, sm);
#pragma unroll
      for (int s = 0; s < E; ++s) {
        if (!freeb[s]) continue;
        if (!sel.exact ? key[s] >= sel.lo : key[s] > sel.lo) top += huber(a[s], M);
      }
      if (sel.exact && sel.take > 0 && threadIdx.x == 0)
        top += (double)sel.take * huber(bitsd(sel.lo), M);
    }
  }
  return bsum(z1 + top, sm);
}

}  // namespace cgl

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
  double hb[kMaxHead];      // head breakpoints huber_prox(rho, hu_i, M)
  int hidx[kMaxHead + 1];
  double tmp[kMaxHead];
  double redd[kProxWaves * 4];
  double fsw[kProxWaves];  // per-wave partial sums a caller keeps across the prox
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
struct ArgMax {
  double v;
  int i;
  int pad;
};
struct OpArgMax {
  __device__ __forceinline__ ArgMax operator()(ArgMax a, ArgMax b) const {
    return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a;
  }
};
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  const ArgMax r = wave_reduce(ArgMax{v, i, 0}, ArgMax{-HUGE_VAL, INT_MAX, 0}, OpArgMax());
  v = r.v;
  i = r.i;
}

// The K largest active keys (K <= kWaveSel, K <= number of active keys), sorted decreasingly
// (ties: smaller index first), into sm.hu[0..K) / sm.hidx[0..K). key(s) is the key of this
// thread's element s (index s * kProxThreads + tid), act bit s whether it takes part; keys are
// recomputed from the caller's registers on every scan instead of being held in another array.
template <int E, typename KeyF>
__device__ __forceinline__ void block_topk(KeyF key, uint32_t act, int K, ProxSmem& sm) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  uint32_t avail = act;
  for (int r = 0; r < K; ++r) {
    double bv = -1.0;  // keys are >= 0
    int bi = INT_MAX;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const double ks = key(s);
      // elements are visited in increasing index, so a strict > keeps the smaller index on ties
      if (((avail >> s) & 1u) && ks > bv) {
        bv = ks;
        bi = s * kProxThreads + (int)threadIdx.x;
      }
    }
    wave_argmax(bv, bi);
    if (bi != INT_MAX && (bi & (kProxThreads - 1)) == (int)threadIdx.x)
      avail &= ~(1u << (bi / kProxThreads));
    if (lane == 0) {
      sm.cand_v[wid * kWaveSel + r] = bv;
      sm.cand_i[wid * kWaveSel + r] = bi;
    }
  }
  __syncthreads();
  if (wid == 0) {
    // each wave's K candidates are sorted (value desc, index asc): merge the kProxWaves lists,
    // lane q holding the current head of list q (element indices are unique across waves)
    const int q = lane;
    int pos = 0;
    double hv = -1.0;
    int hi = INT_MAX;
    if (q < kProxWaves) {
      hv = sm.cand_v[q * kWaveSel];
      hi = sm.cand_i[q * kWaveSel];
    }
    for (int r = 0; r < K; ++r) {
      double wv = hv;
      int wi = hi;
      wave_argmax(wv, wi);
      if (lane == 0) {
        sm.hu[r] = wv;
        sm.hidx[r] = wi;
      }
      if (q < kProxWaves && wi != INT_MAX && hi == wi) {
        ++pos;
        if (pos < K) {
          hv = sm.cand_v[q * kWaveSel + pos];
          hi = sm.cand_i[q * kWaveSel + pos];
        } else {
          hv = -1.0;
          hi = INT_MAX;
        }
      }
    }
  }
  __syncthreads();
}

// A node's record of the winners of its last selection (rec[0] = K, rec[1..K] = element
// indices; 65 ints), read ahead of the selection so that the load's latency is spent elsewhere:
// k0 = rec[0] and, for the first 64 threads, idx = rec[1 + threadIdx.x].
struct WarmPrev {
  int* rec;
  int k0;
  int idx;
};
__device__ __forceinline__ WarmPrev warm_prev(int* rec) {
  WarmPrev w{rec, -1, 0};
  if (rec != nullptr) {
    w.k0 = rec[0];
    if (threadIdx.x < 64) w.idx = rec[1 + threadIdx.x];
  }
  return w;
}

// Warm-started selection of the K largest (the same order as block_topk: value desc, index asc)
// from the K winners of the previous call on this node (wp). Their current values give a
// threshold tau = min over them, and at least K elements have a value >= tau, so the K largest
// all lie in {value >= tau}; those candidates (at most kWarmCap) are ranked exactly. uv[j]: the
// value of element j (ABS: its magnitude) for every j < E * kProxThreads (an LDS array indexed
// by element). Returns false, having written nothing in sm.hu / sm.hidx, when there is no usable
// history or too many candidates; the caller then runs block_topk. On success the winners are
// stored back into the record for the next call.
constexpr int kWarmCap = 256;
template <int E, bool ABS>
__device__ __noinline__ bool block_topk_warm(const double* uv, uint32_t act, int K, WarmPrev wp,
                                             ProxSmem& sm) {
  if (wp.rec == nullptr || wp.k0 != K) return false;  // uniform
  const int tid = threadIdx.x;
  auto val = [&](int j) { return ABS ? fabs(uv[j]) : uv[j]; };
  if (tid < 64) {
    double t = tid < K ? val(wp.idx) : HUGE_VAL;
    t = wave_reduce(t, HUGE_VAL, OpMin());
    if (tid == 0) {
      sm.b_dbl[0] = t;
      sm.b_int[0] = 0;
    }
  }
  __syncthreads();
  const double tau = sm.b_dbl[0];
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int j = s * kProxThreads + tid;
    if (!((act >> s) & 1u)) continue;
    const double v = val(j);
    if (v >= tau) {
      const int slot = atomicAdd(&sm.b_int[0], 1);
      if (slot < kWarmCap) {
        sm.cand_v[slot] = v;
        sm.cand_i[slot] = j;
      }
    }
  }
  __syncthreads();
  const int c = sm.b_int[0];
  if (c > kWarmCap || c < K) return false;  // uniform
  for (int q = tid; q < c; q += blockDim.x) {
    const double v = sm.cand_v[q];
    const int i = sm.cand_i[q];
    int rank = 0;
    for (int r = 0; r < c; ++r) {
      const double w = sm.cand_v[r];
      rank += (w > v || (w == v && sm.cand_i[r] < i)) ? 1 : 0;
    }
    if (rank < K) {
      sm.hu[rank] = v;
      sm.hidx[rank] = i;
    }
  }
  __syncthreads();
  if (tid < K) wp.rec[1 + tid] = sm.hidx[tid];
  return true;
}

// Record the K winners of a block_topk call for the next warm start.
__device__ __forceinline__ void topk_remember(int* prev, int K, const ProxSmem& sm) {
  if (prev == nullptr) return;
  if (threadIdx.x < K) prev[1 + threadIdx.x] = sm.hidx[threadIdx.x];
  if (threadIdx.x == 0) prev[0] = K;
}

// Result of a descending radix selection: selected = key > lo, plus `take` of the keys == lo
// when `exact`; when !exact, selected = key >= lo (and the count is exactly the requested one).
struct Select {
  uint64_t lo;
  bool exact;
  int take;
};

// need-th largest among active keys (1 <= need <= number of active keys). Byte-wise radix.
template <int E, typename KeyF>
__device__ __forceinline__ Select radix_select_desc(KeyF key, uint32_t act, int need, ProxSmem& sm) {
  uint64_t o = 0, a = ~(uint64_t)0;
#pragma unroll
  for (int s = 0; s < E; ++s)
    if ((act >> s) & 1u) { o |= key(s); a &= key(s); }
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
      const uint64_t ks = key(s);
      if (((act >> s) & 1u) && (hs >= 64 || (ks >> hs) == (prefix >> hs)))
        atomicAdd(&sm.cnt[(ks >> shift) & 255], 1u);
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
      cand = wave_reduce(cand, INT_MIN, OpMax());
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
// of H: hb_i = huber_prox(rho, hu_i, M) (precomputed) and M. Every wave evaluates it (no
// barrier needed).
__device__ double psi_root(const double* hu, const double* hb, int kh, double vlo, double m,
                           double S, double rho, double M) {
  const int lane = threadIdx.x & 63;
  double a = vlo, b = HUGE_VAL;
  for (int base = 0; base <= kh; base += 64) {
    const int i = base + lane;
    if (i <= kh) {
      const double pt = (i < kh) ? hb[i] : M;
      if (pt > vlo) {
        const double ps = head_part(hu, kh, pt, rho, M) - (S - m * pt);
        if (ps <= 0.0) a = fmax(a, pt);
        else b = fmin(b, pt);
      }
    }
  }
  a = wave_reduce(a, -HUGE_VAL, OpMax());
  b = wave_reduce(b, HUGE_VAL, OpMin());
  // membership of the head and the regime of min(v, M) are constant on (a, b)
  const double mid = isinf(b) ? a + fmax(1.0, fabs(a)) : 0.5 * (a + b);
  double nh = 0.0, sh = 0.0;
  for (int i = 0; i < kh; ++i) {
    if (hb[i] < mid) { nh += 1.0; sh += hu[i]; }
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
template <int E, typename UF>
__device__ __forceinline__ double tail_root(UF u, uint32_t tail, const double* hu, const double* hb, int kh,
                           double v0, double rho, double M, ProxSmem& sm) {
  double v = v0 > 0.0 ? v0 : 0.0;
  double m_prev = -1.0;
  bool checked_start = v == 0.0;
  for (int it = 0; it < 4096; ++it) {
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const double us = u(s);
      if (((tail >> s) & 1u) && us > v) { acc[0] += 1.0; acc[1] += us; }
    }
    block_sum_n<2>(acc, sm);
    const double m = acc[0], S = acc[1];
    if (!checked_start) {
      checked_start = true;
      if (head_part(hu, kh, v, rho, M) - (S - m * v) > 0.0) {
        // hint above v*: the members at the hint are a subset of those at any v below it, so
        // the root with this set fixed, searched from 0, is a lower bound on v* (and close to it
        // when the hint is)
        v = psi_root(hu, hb, kh, 0.0, m, S, rho, M);
        continue;
      }
    }
    if (m == m_prev) break;  // the member set did not change: v is the root
    v = psi_root(hu, hb, kh, v, m, S, rho, M);
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

// Class codes of a thread's E elements, 2 bits each (element s at bits 2s, 2s + 1).
__device__ __forceinline__ int cls_at(uint64_t cb, int s) { return (int)((cb >> (2 * s)) & 3u); }
template <int E>
__device__ __forceinline__ uint32_t cls_mask(uint64_t cb, int c) {
  uint32_t m = 0;
#pragma unroll
  for (int s = 0; s < E; ++s) m |= (cls_at(cb, s) == c ? 1u : 0u) << s;
  return m;
}

// Node prox. U(s): u = rho |w| of this thread's element s (index s * kProxThreads + tid), read
// from wherever the caller keeps it (registers, or a per-thread LDS slice); neg bit s: w < 0.
// cb: packed class codes (CLS_*); kp = k - |Z1| (>= 0); nfree = |F|; vhint: previous v* (0 if
// none). The result is handed to out(s, beta_s) once, element by element, at the end.
template <int E, typename UF, typename OutF>
__device__ __forceinline__ ProxOut node_prox(UF U, uint32_t neg, uint64_t cb, int kp, int nfree, double rho,
                             double M, double vhint, OutF out, ProxSmem& sm,
                             const double* uv = nullptr, WarmPrev prev = WarmPrev{nullptr, -1, 0}) {
  const uint32_t fm = cls_mask<E>(cb, CLS_FREE);
  auto sgn = [&](int s, double mag) { return ((neg >> s) & 1u) ? -mag : mag; };
  // Z1 coordinates: ridge-and-clip rho w / (1 + rho) clipped to [-M, M]
  auto z1beta = [&](int s) { return sgn(s, fmin(U(s) / (1.0 + rho), M)); };
  ProxOut res;
  res.vstar = 0.0;
  if (kp <= 0 || nfree == 0 || kp >= nfree) {
    // F pinned to zero (no budget left) or empty; or every free coordinate can take z = 1
    // (ridge-and-clip, g = 1/2 ||beta||^2)
    const bool all_in = kp > 0 && nfree > 0;
    double sq = 0.0;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int c = cls_at(cb, s);
      double b = 0.0;
      if (c == CLS_ONE || (c == CLS_FREE && all_in)) b = z1beta(s);
      out(s, b);
      sq += b * b;
    }
    res.gval = 0.5 * bsum(sq, sm);
    return res;
  }
  // ---- head: the kp largest u over F (sorted into sm.hu), and the largest tail value
  uint32_t head = 0;
  double umax_tail;
  if (kp + 1 <= kWaveSel) {
    // uv: the u values indexed by element (for the warm start); prev: the last call's winners
    if (uv == nullptr || !block_topk_warm<E, false>(uv, fm, kp + 1, prev, sm)) {
      block_topk<E>(U, fm, kp + 1, sm);
      topk_remember(prev.rec, kp + 1, sm);
    }
    const double tv = sm.hu[kp - 1];
    const int ti = sm.hidx[kp - 1];
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int j = s * kProxThreads + (int)threadIdx.x;
      const double us = U(s);
      head |= (((fm >> s) & 1u) && (us > tv || (us == tv && j <= ti)) ? 1u : 0u) << s;
    }
    umax_tail = sm.hu[kp];
  } else {
    auto K = [&](int s) { return dbits(U(s)); };
    const Select sel = radix_select_desc<E>(K, fm, kp, sm);
    if (threadIdx.x == 0) { sm.head_fill = 0; sm.ties_left = sel.exact ? sel.take : 0; }
    __syncthreads();
    double tmax = -1.0;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      if (!((fm >> s) & 1u)) continue;
      const uint64_t ks = K(s);
      bool h;
      if (!sel.exact) h = ks >= sel.lo;
      else if (ks > sel.lo) h = true;
      else if (ks == sel.lo) h = atomicSub(&sm.ties_left, 1) > 0;
      else h = false;
      if (h) {
        head |= 1u << s;
        sm.hu[atomicAdd(&sm.head_fill, 1)] = U(s);
      } else {
        tmax = fmax(tmax, U(s));
      }
    }
    __syncthreads();
    sort_head_desc(kp, sm);
    umax_tail = bmax(tmax, sm);
  }
  // ---- v*: head breakpoints huber_prox(rho, hu_i, M) once, then the root search
  for (int i = threadIdx.x; i < kp; i += blockDim.x) sm.hb[i] = huber_prox(rho, sm.hu[i], M);
  __syncthreads();
  const uint32_t tail = fm & ~head;
  double vstar;
  if (sm.hb[kp - 1] >= umax_tail) {
    vstar = umax_tail;  // no isotonic violation at the junction: no pooled block
  } else {
    vstar = tail_root<E>(U, tail, sm.hu, sm.hb, kp, vhint, rho, M, sm);
  }
  res.vstar = vstar;
  // ---- assemble beta; |beta_F| total and Z1 squares in one reduction
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int s = 0; s < E; ++s) {
    double b = 0.0;
    if ((fm >> s) & 1u) {
      const double us = U(s);
      const double c = ((head >> s) & 1u) ? huber_prox(rho, us, M) : 0.0;
      const double t = us - fmax(c, vstar);
      const double mag = t > 0.0 ? t / rho : 0.0;
      b = mag > 0.0 ? sgn(s, mag) : 0.0;
      acc[0] += mag;
    } else if (cls_at(cb, s) == CLS_ONE) {
      b = z1beta(s);
      acc[1] += b * b;
    }
    out(s, b);
  }
  // head magnitudes in sorted order (|beta| is monotone in u)
  for (int i = threadIdx.x; i < kp; i += blockDim.x) {
    const double uh = sm.hu[i];
    const double t = uh - fmax(sm.hb[i], vstar);
    sm.tmp[i] = t > 0.0 ? t / rho : 0.0;
  }
  block_sum_n<2>(acc, sm);
  if (threadIdx.x == 0) sm.b_dbl[3] = alg2_from_sorted(sm.tmp, kp, kp, acc[0]);
  __syncthreads();
  res.gval = 0.5 * acc[1] + sm.b_dbl[3];
  __syncthreads();
  return res;
}

// g_node*(a) = sum_{Z1} H_M(a_j) + TopSum_{kp}(H_M(a_F))  (Lemma 2, separable sum rule), with
// |a_j| = A(j) / div (A(s): the magnitude of this thread's element s before the division).
// H_M is increasing in |a| and the division is monotone, so the top kp of H_M(a_F) are found
// on A directly and only the selected values are divided.
template <int E, typename AF>
__device__ __forceinline__ double gstar_node(AF A, double div, uint64_t cb, int kp, int nfree, double M,
                             ProxSmem& sm, const double* av = nullptr,
                             WarmPrev prev = WarmPrev{nullptr, -1, 0}) {
  const uint32_t fm = cls_mask<E>(cb, CLS_FREE);
  double z1 = 0.0;
#pragma unroll
  for (int s = 0; s < E; ++s)
    if (cls_at(cb, s) == CLS_ONE) z1 += huber(A(s) / div, M);
  double top = 0.0;
  if (kp > 0 && nfree > 0) {
    if (kp >= nfree) {
#pragma unroll
      for (int s = 0; s < E; ++s)
        if ((fm >> s) & 1u) top += huber(A(s) / div, M);
    } else if (kp <= kWaveSel) {
      // av: signed values indexed by element (A = |av|) for the warm start
      if (av == nullptr || !block_topk_warm<E, true>(av, fm, kp, prev, sm)) {
        block_topk<E>(A, fm, kp, sm);
        topk_remember(prev.rec, kp, sm);
      }
      if (threadIdx.x == 0)
        for (int r = 0; r < kp; ++r) top += huber(sm.hu[r] / div, M);
    } else {
      auto K = [&](int s) { return dbits(A(s)); };
      const Select sel = radix_select_desc<E>(K, fm, kp, sm);
#pragma unroll
      for (int s = 0; s < E; ++s) {
        if (!((fm >> s) & 1u)) continue;
        const uint64_t ks = K(s);
        if (!sel.exact ? ks >= sel.lo : ks > sel.lo) top += huber(A(s) / div, M);
      }
      if (sel.exact && sel.take > 0 && threadIdx.x == 0)
        top += (double)sel.take * huber(bitsd(sel.lo) / div, M);
    }
  }
  return bsum(z1 + top, sm);
}

// Per-thread working values of the prox kernels: element s of thread t at s * kProxThreads + t
// of an LDS array (private to the thread: no barrier needed) for s < kLdsElems, in registers
// beyond (E > kLdsElems: the first kLdsElems in LDS, the rest in registers). Keeps register
// pressure low enough for 1024-thread workgroups.
constexpr int kLdsElems = 16;
template <int E>
struct ProxVals {
  static constexpr bool lds = E <= kLdsElems;              // every value in the LDS slice
  static constexpr int nl = E < kLdsElems ? E : kLdsElems;  // values in the LDS slice
  static constexpr int nr = E - nl;                          // values in registers
  double* sl;                                                // LDS slice base (nl * kProxThreads)
  double reg[nr > 0 ? nr : 1];
  __device__ __forceinline__ void set(int s, double v) {
    if (s < nl) sl[s * kProxThreads + threadIdx.x] = v;
    else reg[s - nl] = v;
  }
  __device__ __forceinline__ double get(int s) const {
    if (s < nl) return sl[s * kProxThreads + threadIdx.x];
    return reg[s - nl];
  }
};

}  // namespace cgl

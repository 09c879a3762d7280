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
// On the GPU the head is found by a byte-wise radix select on the FP64 bit patterns of u (they
// order like the values for u >= 0), and v* by a radix search over the tail bit patterns that
// keeps FP64 per-bin counts and sums, so phi can be evaluated exactly at every bin edge; the
// last interval is solved in closed form. No sort of the p entries is needed.
#pragma once

#include "common.h"

namespace cgl {

constexpr int kProxThreads = 1024;
constexpr int kProxWaves = kProxThreads / kWave;
constexpr int kMaxHead = 256;  // supports k' <= 256

enum : uint8_t { CLS_FREE = 0, CLS_ZERO = 1, CLS_ONE = 2, CLS_PAD = 3 };

struct ProxSmem {
  uint32_t cnt[256];
  double sum[256];
  double hu[kMaxHead];  // head u values, sorted decreasingly after gather
  double tmp[kMaxHead];
  double redd[kProxWaves * 2];
  uint64_t redu[kProxWaves];
  int redi[kProxWaves];
  int head_fill;
  int ties_left;
  // broadcast slots
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

// Result of a descending selection: selected = key > lo, plus `take` of the keys == lo when
// `exact`; when !exact, selected = key >= lo (and the count is exactly the requested one).
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
      int suf = wave_suffix_incl(loc);
      int excl = suf - loc;  // bins of higher lanes
      int best = -1, above = 0, binc = 0;
      int run = excl;
#pragma unroll
      for (int i = 3; i >= 0; --i) {
        int incl = run + c[i];
        if (best < 0 && incl >= remaining) { best = lane * 4 + i; above = run; binc = c[i]; }
        run = incl;
      }
      // highest bin whose suffix reaches `remaining`
      int cand = best;
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

__device__ __forceinline__ bool selected(uint64_t k, const Select& sel, int& tie_slot_out) {
  tie_slot_out = -1;
  if (!sel.exact) return k >= sel.lo;
  if (k > sel.lo) return true;
  return false;  // ties handled by the caller
}

// head part of phi: sum over head values hu[0..kh) of [(v - u) + rho min(v, M)]_+
__device__ __forceinline__ double head_part(const double* hu, int kh, double v, double rho,
                                            double M) {
  double acc = 0.0;
  const double pen = rho * fmin(v, M);
  for (int i = 0; i < kh; ++i) {
    double t = (v - hu[i]) + pen;
    acc += t > 0.0 ? t : 0.0;
  }
  return acc;
}

// Closed form of the root of phi on an interval where the tail members (m, S) are fixed:
// members of the head are those with huber_prox(rho, u) < v; solve at the membership of `mid`.
__device__ __forceinline__ double solve_linear_piece(const double* hu, int kh, double mid, int m,
                                                     double S, double rho, double M) {
  int nh = 0;
  double sh = 0.0;
  for (int i = 0; i < kh; ++i) {
    if (huber_prox(rho, hu[i], M) < mid) { ++nh; sh += hu[i]; }
  }
  if (mid <= M) {
    double den = (double)m + (double)nh * (1.0 + rho);
    return den > 0.0 ? (S + sh) / den : mid;
  }
  double den = (double)(m + nh);
  return den > 0.0 ? (S + sh - rho * M * (double)nh) / den : mid;
}

// Exact root of phi on [lo, hi] with tail members (m, S) fixed. Breakpoints inside come from
// the head (huber_prox values) and from M. Evaluated by wave 0; result broadcast.
__device__ double final_root(const double* hu, int kh, double lo, double hi, int m, double S,
                             double rho, double M, ProxSmem& sm) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    // largest point with phi <= 0 and smallest point with phi > 0 among {lo, hi, M, c_i}
    double a = lo, b = hi;
    const int npts = kh + 1;
    for (int base = 0; base < npts; base += 64) {
      int i = base + lane;
      if (i < npts) {
        double pt = (i < kh) ? huber_prox(rho, hu[i], M) : M;
        if (pt > lo && pt < hi) {
          double ph = head_part(hu, kh, pt, rho, M) - (S - (double)m * pt);
          if (ph <= 0.0) a = fmax(a, pt);
          else b = fmin(b, pt);
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a = fmax(a, __shfl_xor(a, off, kWave));
      b = fmin(b, __shfl_xor(b, off, kWave));
    }
    if (lane == 0) {
      double mid = 0.5 * (a + b);
      double v = solve_linear_piece(hu, kh, mid, m, S, rho, M);
      v = fmin(fmax(v, a), b);
      sm.b_dbl[0] = v;
    }
  }
  __syncthreads();
  double v = sm.b_dbl[0];
  __syncthreads();
  return v;
}

// v* for the tail (act = free and not head), given the sorted head values in sm.hu[0..kh).
// Returns v*. umax_tail: largest tail u (phi(umax_tail) >= 0).
template <int E>
__device__ double tail_root(const double (&u)[E], const bool (&act)[E], int kh, double rho,
                            double M, ProxSmem& sm) {
  uint64_t key[E];
  uint64_t o = 0, a = ~(uint64_t)0;
  double umax = 0.0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    key[s] = dbits(u[s]);
    if (act[s]) { o |= key[s]; a &= key[s]; umax = fmax(umax, u[s]); }
  }
  o = bor(o, sm);
  a = band(a, sm);
  umax = bmax(umax, sm);
  int m_above = 0;
  double s_above = 0.0;
  double lo = 0.0, hi = umax;
  const uint64_t diff = o ^ a;
  if (diff == 0) {
    // every tail value equals umax: members iff v* < umax
    int c = 0;
#pragma unroll
    for (int s = 0; s < E; ++s) c += act[s] ? 1 : 0;
    c = bsum_i(c, sm);
    double ph = head_part(sm.hu, kh, umax, rho, M);
    if (ph > 0.0) return final_root(sm.hu, kh, 0.0, umax, c, (double)c * umax, rho, M, sm);
    return umax;  // phi(umax) = 0 with no tail member: no pooled tail
  }
  const int hb = 63 - __clzll(diff);
  int shift = (hb >> 3) << 3;
  uint64_t prefix = (shift + 8 >= 64) ? 0 : (a & ~((((uint64_t)1) << (shift + 8)) - 1));
  const int lane = threadIdx.x & 63;
  bool first = true;
  for (;;) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) { sm.cnt[i] = 0; sm.sum[i] = 0.0; }
    __syncthreads();
    const int hs = shift + 8;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      if (act[s] && (hs >= 64 || (key[s] >> hs) == (prefix >> hs))) {
        const int bin = (int)((key[s] >> shift) & 255);
        atomicAdd(&sm.cnt[bin], 1u);
        atomicAdd(&sm.sum[bin], u[s]);
      }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      int c[4];
      double sv[4];
      int loc = 0;
      double locs = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        c[i] = (int)sm.cnt[lane * 4 + i];
        sv[i] = sm.sum[lane * 4 + i];
        loc += c[i];
        locs += sv[i];
      }
      const int sufc = wave_suffix_incl(loc);
      const double sufs = wave_suffix_incl(locs);
      int runc = sufc - loc;      // bins above this lane's four
      double runs = sufs - locs;
      int best = -1;
      int best_above_c = 0;
      double best_above_s = 0.0;
#pragma unroll
      for (int i = 3; i >= 0; --i) {
        const int b = lane * 4 + i;
        const int ic = runc + c[i];
        const double is = runs + sv[i];
        const uint64_t ekey = prefix | (((uint64_t)b) << shift);
        const double tau = bitsd(ekey);
        // only edges inside [lo, hi] order like their bins: a digit that covers the sign bit
        // would otherwise decode to negative edges, and NaN / inf edges are meaningless
        const bool eligible = (ekey >> 63) == 0 && tau <= hi;
        const double ph = head_part(sm.hu, kh, tau, rho, M) -
                          ((s_above + is) - (double)(m_above + ic) * tau);
        if (best < 0 && eligible && ph <= 0.0) {
          best = b; best_above_c = runc; best_above_s = runs;
        }
        runc = ic;
        runs = is;
      }
      int cand = best;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) cand = max(cand, __shfl_xor(cand, off, kWave));
      if (lane == 0 && cand < 0) {
        sm.b_int[0] = -1;
        sm.b_int[1] = sufc;  // lane 0 holds the total
        sm.b_dbl[1] = sufs;
      }
      if (cand >= 0 && best == cand) {
        sm.b_int[0] = best;
        sm.b_int[1] = best_above_c;
        sm.b_dbl[1] = best_above_s;
        sm.b_int[2] = c[best & 3];
        sm.b_dbl[2] = sv[best & 3];
      }
    }
    __syncthreads();
    const int b = sm.b_int[0];
    const int above_c = sm.b_int[1];
    const double above_s = sm.b_dbl[1];
    const int binc = sm.b_int[2];
    const double bins = sm.b_dbl[2];
    __syncthreads();
    if (b < 0) {
      // phi > 0 at the bottom of the range: every candidate is a member (first pass only)
      const double top = bitsd(prefix);
      (void)first;
      return final_root(sm.hu, kh, lo, fmin(top, hi), m_above + above_c, s_above + above_s,
                        rho, M, sm);
    }
    first = false;
    m_above += above_c;
    s_above += above_s;
    lo = bitsd(prefix | (((uint64_t)b) << shift));
    if (b < 255) {
      const uint64_t nkey = prefix | (((uint64_t)(b + 1)) << shift);
      if ((nkey >> 63) == 0) hi = fmin(hi, bitsd(nkey));
    }
    if (binc == 0) return final_root(sm.hu, kh, lo, hi, m_above, s_above, rho, M, sm);
    if (binc == 1 || shift == 0) {
      const double uc = (binc == 1) ? bins : bitsd(prefix | (uint64_t)b);
      const double ph = head_part(sm.hu, kh, uc, rho, M) - (s_above - (double)m_above * uc);
      if (ph <= 0.0) return final_root(sm.hu, kh, uc, hi, m_above, s_above, rho, M, sm);
      return final_root(sm.hu, kh, lo, uc, m_above + binc, s_above + bins, rho, M, sm);
    }
    prefix |= ((uint64_t)b) << shift;
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
  double gval;  // g_node(beta)
  double vstar; // pooled value (diagnostic)
};

// Node prox in registers. w: element s of this thread is index j = s * blockDim + tid.
// cls: CLS_*; kp = k - |Z1| (>= 0); nfree = |F|. beta receives the result.
template <int E>
__device__ ProxOut node_prox(const double (&w)[E], const uint8_t (&cls)[E], int kp, int nfree,
                             double rho, double M, double (&beta)[E], ProxSmem& sm) {
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
  if (kp <= 0 || nfree == 0) {
    // F pinned to zero (no budget) or empty
    out.gval = 0.5 * bsum(z1sq, sm);
    return out;
  }
  if (kp >= nfree) {
    // every free coordinate can take z = 1: ridge-and-clip, g = 1/2 ||beta||^2
    double sq = z1sq;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      if (freeb[s]) {
        double b = fmin(u[s] / (1.0 + rho), M);
        b = copysign(b, w[s]);
        if (w[s] == 0.0) b = 0.0;
        beta[s] = b;
        sq += b * b;
      }
    }
    out.gval = 0.5 * bsum(sq, sm);
    return out;
  }
  // ---- head: top-kp of u over F
  uint64_t key[E];
#pragma unroll
  for (int s = 0; s < E; ++s) key[s] = dbits(u[s]);
  const Select sel = radix_select_desc<E>(key, freeb, kp, sm);
  if (threadIdx.x == 0) { sm.head_fill = 0; sm.ties_left = sel.exact ? sel.take : 0; }
  __syncthreads();
  bool head[E];
#pragma unroll
  for (int s = 0; s < E; ++s) {
    bool h = false;
    if (freeb[s]) {
      if (!sel.exact) h = key[s] >= sel.lo;
      else if (key[s] > sel.lo) h = true;
      else if (key[s] == sel.lo) h = atomicSub(&sm.ties_left, 1) > 0;
    }
    head[s] = h;
    if (h) {
      const int slot = atomicAdd(&sm.head_fill, 1);
      sm.hu[slot] = u[s];
    }
  }
  __syncthreads();
  sort_head_desc(kp, sm);
  // ---- tail root
  bool tail[E];
#pragma unroll
  for (int s = 0; s < E; ++s) tail[s] = freeb[s] && !head[s];
  const double vstar = tail_root<E>(u, tail, kp, rho, M, sm);
  out.vstar = vstar;
  // ---- assemble beta, |beta_F| total, Z1 squares
  double absF = 0.0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    if (freeb[s]) {
      const double c = head[s] ? huber_prox(rho, u[s], M) : 0.0;
      const double t = u[s] - fmax(c, vstar);
      double mag = t > 0.0 ? t / rho : 0.0;
      beta[s] = copysign(mag, w[s]);
      if (mag == 0.0) beta[s] = 0.0;
      absF += mag;
    }
  }
  // head magnitudes in sorted order (monotone in u)
  for (int i = threadIdx.x; i < kp; i += blockDim.x) {
    const double uh = sm.hu[i];
    const double t = uh - fmax(huber_prox(rho, uh, M), vstar);
    sm.tmp[i] = t > 0.0 ? t / rho : 0.0;
  }
  const double sF = bsum(absF, sm);
  const double sq1 = bsum(z1sq, sm);
  if (threadIdx.x == 0) sm.b_dbl[3] = alg2_from_sorted(sm.tmp, kp, kp, sF);
  __syncthreads();
  out.gval = 0.5 * sq1 + sm.b_dbl[3];
  __syncthreads();
  return out;
}

// g_node*(a) = sum_{Z1} H_M(a_j) + TopSum_{kp}(H_M(a_F))  (Lemma 2, separable sum rule).
template <int E>
__device__ double gstar_node(const double (&a)[E], const uint8_t (&cls)[E], int kp, int nfree,
                             double M, ProxSmem& sm) {
  double z1 = 0.0;
  bool freeb[E];
  uint64_t key[E];
#pragma unroll
  for (int s = 0; s < E; ++s) {
    freeb[s] = cls[s] == CLS_FREE;
    key[s] = dbits(fabs(a[s]));
    if (cls[s] == CLS_ONE) z1 += huber(a[s], M);
  }
  double top = 0.0;
  if (kp > 0 && nfree > 0) {
    if (kp >= nfree) {
#pragma unroll
      for (int s = 0; s < E; ++s)
        if (freeb[s]) top += huber(a[s], M);
    } else {
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

// Node prox for long vectors (p above what one workgroup holds in registers or LDS): the same
// structure as node_prox in prox.h (Lemma 3 and Alg. 1: one pooled block at the head/tail
// junction, its value v* the root of phi), with every block-wide step streaming the vector from
// memory instead of holding it per thread. One 1024-thread workgroup per vector; element j is
// visited by thread j mod 1024 in pass order j = tid, tid + 1024, ...
//
// Head selection: the k' largest u = rho |w_F| (ties: smaller index first). The k'-th largest of
// the threads' own maxima is a lower bound tau on the k'-th largest u (at least k' elements, the
// maxima above it, reach it), so the head lies in {u >= tau}; those candidates (usually a few
// times k') are gathered into LDS and ranked exactly. When they do not fit, a byte-wise radix
// selection over all elements finds the k'-th largest key and a search over the index finds
// which of the tied elements come first.
#include <limits.h>

#include "common.h"
#include "kernels.h"
#include "prox.h"
#include "solver.h"

namespace cgl {

constexpr int kPagedCand = 2048;  // candidates ranked in LDS

struct PagedSmem {
  double cv[kPagedCand];
  int ci[kPagedCand];
  int ccount;
  double tmax;
};

__global__ __launch_bounds__(1024) void k_prox_paged(const double* __restrict__ w, int64_t w_ld,
                                                     const uint8_t* __restrict__ cls_all,
                                                     int64_t cls_ld, int64_t p, double rho,
                                                     double M, NodeDev* __restrict__ st_all,
                                                     double* __restrict__ b_all,
                                                     int64_t b_ld) {
  __shared__ ProxSmem sm;
  __shared__ PagedSmem pm;
  const int node = blockIdx.x;
  NodeDev* st = st_all + node;
  const int tid = threadIdx.x;
  const double* wn = w + (int64_t)node * w_ld;
  const uint8_t* cn = cls_all + (int64_t)node * cls_ld;
  double* bn = b_all + (int64_t)node * b_ld;
  const int kp = st->kp;
  const int nfree = st->nfree;
  auto U = [&](int64_t j) { return rho * fabs(wn[j]); };
  auto sgn = [&](int64_t j, double mag) { return wn[j] < 0.0 ? -mag : mag; };
  auto z1beta = [&](int64_t j) { return sgn(j, fmin(U(j) / (1.0 + rho), M)); };

  if (kp <= 0 || nfree == 0 || kp >= nfree) {
    // F pinned to zero or empty, or every free coordinate within the budget (ridge-and-clip)
    const bool all_in = kp > 0 && nfree > 0;
    double sq = 0.0;
    for (int64_t j = tid; j < p; j += kProxThreads) {
      const int c = cn[j];
      double b = 0.0;
      if (c == CLS_ONE || (c == CLS_FREE && all_in)) b = z1beta(j);
      bn[j] = b;
      sq += b * b;
    }
    const double g = 0.5 * bsum(sq, sm);
    if (tid == 0) {
      st->g_new = g;
      st->vstar = 0.0;
    }
    return;
  }

  // ---- tau: the kp-th largest of the threads' maxima over F (0 when fewer threads have one)
  double tm = -1.0;
  for (int64_t j = tid; j < p; j += kProxThreads)
    if (cn[j] == CLS_FREE) tm = fmax(tm, U(j));
  double tau = 0.0;
  {
    auto K = [&](int) { return dbits(tm); };
    const uint32_t act = tm >= 0.0 ? 1u : 0u;
    const int nact = bsum_i((int)act, sm);
    if (nact >= kp) tau = bitsd(radix_select_desc<1>(K, act, kp, sm).lo);
  }
  // ---- candidates u >= tau into LDS; the largest value below them
  if (tid == 0) pm.ccount = 0;
  __syncthreads();
  double below = -1.0;
  for (int64_t j = tid; j < p; j += kProxThreads) {
    if (cn[j] != CLS_FREE) continue;
    const double u = U(j);
    if (u >= tau) {
      const int slot = atomicAdd(&pm.ccount, 1);
      if (slot < kPagedCand) {
        pm.cv[slot] = u;
        pm.ci[slot] = (int)j;
      }
    } else {
      below = fmax(below, u);
    }
  }
  below = bmax(below, sm);
  const int cc = pm.ccount;  // read after the barriers of bmax
  // head: sm.hu[0..kp) sorted decreasingly; membership rule by (value, index)
  double cut_v;       // the kp-th largest u
  int64_t cut_j;      // elements with u == cut_v are in the head iff j <= cut_j
  double umax_tail;   // the largest u of the tail
  if (cc <= kPagedCand) {
    // exact rank of every candidate: value desc, index asc
    for (int q = tid; q < cc; q += kProxThreads) {
      const double v = pm.cv[q];
      const int i = pm.ci[q];
      int rank = 0;
      for (int r = 0; r < cc; ++r) {
        const double x = pm.cv[r];
        rank += (x > v || (x == v && pm.ci[r] < i)) ? 1 : 0;
      }
      if (rank <= kp && rank <= kMaxHead) {
        sm.hu[rank] = v;
        sm.hidx[rank] = i;
      }
    }
    __syncthreads();
    cut_v = sm.hu[kp - 1];
    cut_j = sm.hidx[kp - 1];
    umax_tail = cc > kp ? sm.hu[kp] : below;
    __syncthreads();
  } else {
    // radix selection over all free elements, then the index cut among the ties
    auto K = [&](int64_t j) { return dbits(U(j)); };
    uint64_t o = 0, a = ~(uint64_t)0;
    for (int64_t j = tid; j < p; j += kProxThreads)
      if (cn[j] == CLS_FREE) { o |= K(j); a &= K(j); }
    o = bor(o, sm);
    a = band(a, sm);
    uint64_t lo = a;
    int take = kp;  // ties at lo that belong to the head
    bool exact = true;
    const uint64_t diff = o ^ a;
    if (diff != 0) {
      const int hbit = 63 - __clzll(diff);
      int shift = (hbit >> 3) << 3;
      uint64_t prefix = (shift + 8 >= 64) ? 0 : (a & ~((((uint64_t)1) << (shift + 8)) - 1));
      int remaining = kp;
      for (;;) {
        for (int i = tid; i < 256; i += kProxThreads) sm.cnt[i] = 0;
        __syncthreads();
        const int hs = shift + 8;
        for (int64_t j = tid; j < p; j += kProxThreads) {
          if (cn[j] != CLS_FREE) continue;
          const uint64_t ks = K(j);
          if (hs >= 64 || (ks >> hs) == (prefix >> hs)) atomicAdd(&sm.cnt[(ks >> shift) & 255], 1u);
        }
        __syncthreads();
        if (tid < 64) {
          // highest bin whose suffix count reaches `remaining`
          int c4[4];
          int loc = 0;
#pragma unroll
          for (int i = 3; i >= 0; --i) { c4[i] = (int)sm.cnt[tid * 4 + i]; loc += c4[i]; }
          const int suf = wave_suffix_incl(loc);
          int best = -1, above = 0, binc = 0;
          int run = suf - loc;
#pragma unroll
          for (int i = 3; i >= 0; --i) {
            const int incl = run + c4[i];
            if (best < 0 && incl >= remaining) { best = tid * 4 + i; above = run; binc = c4[i]; }
            run = incl;
          }
          const int cand = wave_reduce(best, INT_MIN, OpMax());
          if (best == cand && best >= 0) {
            sm.b_int[0] = best;
            sm.b_int[1] = above;
            sm.b_int[2] = binc;
          }
        }
        __syncthreads();
        const int b = sm.b_int[0], above = sm.b_int[1], binc = sm.b_int[2];
        __syncthreads();
        remaining -= above;
        prefix |= ((uint64_t)b) << shift;
        if (binc == remaining) { lo = prefix; exact = false; break; }
        if (shift == 0) { lo = prefix; take = remaining; break; }
        shift -= 8;
      }
    }
    cut_v = bitsd(lo);
    if (!exact) {
      // exactly kp keys >= lo: the smallest of them is the cut, every tie at it is in the head
      cut_j = INT64_MAX;
    } else {
      // the `take` smallest indices among the keys == lo: cut_j = the take-th one, found by a
      // search over J of count{ j < J : key == lo } >= take
      int64_t lo_j = 0, hi_j = p;  // count(< hi_j) >= take
      while (hi_j - lo_j > 1) {
        const int64_t mid = lo_j + (hi_j - lo_j) / 2;
        int c = 0;
        for (int64_t j = tid; j < mid; j += kProxThreads)
          c += (cn[j] == CLS_FREE && K(j) == lo) ? 1 : 0;
        c = bsum_i(c, sm);
        if (c >= take) hi_j = mid;
        else lo_j = mid;
      }
      cut_j = hi_j - 1;
    }
    // gather the head values (exactly kp) and the largest tail value
    if (tid == 0) sm.head_fill = 0;
    __syncthreads();
    double tmx = -1.0;
    for (int64_t j = tid; j < p; j += kProxThreads) {
      if (cn[j] != CLS_FREE) continue;
      const double u = U(j);
      if (u > cut_v || (u == cut_v && j <= cut_j)) sm.hu[atomicAdd(&sm.head_fill, 1)] = u;
      else tmx = fmax(tmx, u);
    }
    __syncthreads();
    sort_head_desc(kp, sm);
    umax_tail = bmax(tmx, sm);
  }
  auto in_head = [&](int64_t j, double u) { return u > cut_v || (u == cut_v && j <= cut_j); };

  // ---- v*: breakpoints of the head, then the monotone root search over the tail
  for (int i = tid; i < kp; i += kProxThreads) sm.hb[i] = huber_prox(rho, sm.hu[i], M);
  __syncthreads();
  double vstar;
  if (sm.hb[kp - 1] >= umax_tail) {
    vstar = umax_tail;  // no violation at the junction: no pooled block
  } else {
    double v = st->vstar > 0.0 ? st->vstar : 0.0;
    double m_prev = -1.0;
    bool checked_start = v == 0.0;
    for (int it = 0; it < 4096; ++it) {
      double acc[2] = {0.0, 0.0};
      for (int64_t j = tid; j < p; j += kProxThreads) {
        if (cn[j] != CLS_FREE) continue;
        const double u = U(j);
        if (u > v && !in_head(j, u)) { acc[0] += 1.0; acc[1] += u; }
      }
      block_sum_n<2>(acc, sm);
      const double m = acc[0], S = acc[1];
      if (!checked_start) {
        checked_start = true;
        if (head_part(sm.hu, kp, v, rho, M) - (S - m * v) > 0.0) {
          v = psi_root(sm.hu, sm.hb, kp, 0.0, m, S, rho, M);
          continue;
        }
      }
      if (m == m_prev) break;
      v = psi_root(sm.hu, sm.hb, kp, v, m, S, rho, M);
      m_prev = m;
    }
    vstar = v;
  }
  // ---- beta; |beta_F| total and Z1 squares
  double acc[2] = {0.0, 0.0};
  for (int64_t j = tid; j < p; j += kProxThreads) {
    const int c = cn[j];
    double b = 0.0;
    if (c == CLS_FREE) {
      const double u = U(j);
      const double ch = in_head(j, u) ? huber_prox(rho, u, M) : 0.0;
      const double t = u - fmax(ch, vstar);
      const double mag = t > 0.0 ? t / rho : 0.0;
      b = mag > 0.0 ? sgn(j, mag) : 0.0;
      acc[0] += mag;
    } else if (c == CLS_ONE) {
      b = z1beta(j);
      acc[1] += b * b;
    }
    bn[j] = b;
  }
  for (int i = tid; i < kp; i += kProxThreads) {
    const double t = sm.hu[i] - fmax(sm.hb[i], vstar);
    sm.tmp[i] = t > 0.0 ? t / rho : 0.0;
  }
  block_sum_n<2>(acc, sm);
  if (tid == 0) {
    st->g_new = 0.5 * acc[1] + alg2_from_sorted(sm.tmp, kp, kp, acc[0]);
    st->vstar = vstar;
  }
}

void launch_prox_paged(int nodes, const double* w, int64_t w_ld, const uint8_t* cls,
                       int64_t cls_ld, int64_t p, double rho, double M, NodeDev* st, double* b,
                       int64_t b_ld, hipStream_t stream) {
  hipLaunchKernelGGL(k_prox_paged, dim3(nodes), dim3(kProxThreads), 0, stream, w, w_ld, cls,
                     cls_ld, p, rho, M, st, b, b_ld);
}

}  // namespace cgl

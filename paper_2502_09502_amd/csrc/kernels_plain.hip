// Plain FP64 path: FP64 products with X in its stored precision (FP64, FP32 or BF16 values
// upcast exactly), one node per solve. One iteration of Alg. 3 is five launches:
//   k_xt         partial sums of h = X^T grad f(X gamma) over row chunks (HBM pass over X)
//   k_grad_step  h = sum of partials; gamma = beta^t + c (beta^t - beta^{t-1}); w = gamma - h/L
//   k_prox       beta^{t+1} = prox_{g_node/rho}(w); g_node(beta^{t+1}); monitor g_node*(-h/2l2)
//   k_xb         u^{t+1} = X beta^{t+1} and the loss terms f_i(u^{t+1}) (HBM pass over X)
//   k_finish     L^{t+1}, value restart (Alg. 3), best primal, dual bound (Sec. 3.4), stopping
// X gamma is never formed: by linearity X gamma = u^t + c (u^t - u^{t-1}).
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "losses.h"
#include "prox.h"
#include "solver.h"

namespace cgl {

// ------------------------------------------------------------------ vector loads of X

template <typename XT>
struct XVec;
template <>
struct XVec<double> {
  static constexpr int N = 2;
  static __device__ __forceinline__ void load(const double* p, double (&o)[N]) {
    const double2 r = *reinterpret_cast<const double2*>(p);
    o[0] = r.x; o[1] = r.y;
  }
};
template <>
struct XVec<float> {
  static constexpr int N = 4;
  static __device__ __forceinline__ void load(const float* p, double (&o)[N]) {
    const float4 r = *reinterpret_cast<const float4*>(p);
    o[0] = r.x; o[1] = r.y; o[2] = r.z; o[3] = r.w;
  }
};
template <>
struct XVec<uint16_t> {
  static constexpr int N = 8;
  static __device__ __forceinline__ void load(const uint16_t* p, double (&o)[N]) {
    const uint4 r = *reinterpret_cast<const uint4*>(p);
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = (double)__uint_as_float(w[i] << 16);
      o[2 * i + 1] = (double)__uint_as_float(w[i] & 0xFFFF0000u);
    }
  }
};

template <int N>
__device__ __forceinline__ void load_dvec(const double* p, double (&o)[N]) {
#pragma unroll
  for (int i = 0; i < N; i += 2) {
    const double2 r = *reinterpret_cast<const double2*>(p + i);
    o[i] = r.x; o[i + 1] = r.y;
  }
}

__device__ __forceinline__ const double* slot_ptr(const double* base, int64_t stride, int iter,
                                                  int shift) {
  return base + (int64_t)((iter + shift) % 3) * stride;
}
__device__ __forceinline__ double* slot_ptr(double* base, int64_t stride, int iter, int shift) {
  return base + (int64_t)((iter + shift) % 3) * stride;
}

// ------------------------------------------------------------------ u = X beta (+ loss terms)

constexpr int kXbRows = 4;     // rows per wave
constexpr int kXbWaves = 4;    // waves per workgroup

// u = X b. b: p_pad doubles (zero padded), X: n x ldx. If st != nullptr the vectors are ring
// slots selected by st->iter (b = slot iter+1, u = slot iter+1) and the loss terms
// f_i(u_i) are summed per workgroup into loss_part[blockIdx.x].
template <typename XT>
__global__ __launch_bounds__(256) void k_xb(const XT* __restrict__ X, int64_t ldx, int64_t n,
                                            int64_t p_pad, const double* __restrict__ b_base,
                                            int64_t b_stride, double* __restrict__ u_base,
                                            int64_t u_stride, const NodeDev* __restrict__ st,
                                            const double* __restrict__ y, int loss,
                                            double* __restrict__ loss_part) {
  __shared__ double red[kXbWaves];
  if (st != nullptr && st->done) return;
  const int iter = st ? st->iter : 0;
  const double* b = st ? slot_ptr(b_base, b_stride, iter, 1) : b_base;
  double* u = st ? slot_ptr(u_base, u_stride, iter, 1) : u_base;
  constexpr int N = XVec<XT>::N;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t row0 = ((int64_t)blockIdx.x * kXbWaves + wid) * kXbRows;
  double acc[kXbRows];
#pragma unroll
  for (int r = 0; r < kXbRows; ++r) acc[r] = 0.0;
  // Rows past n read row n - 1 (a valid address) and are dropped at the store, so the loop has
  // no branches; the next column chunk of every row is loaded before the current one is used
  // (the last iteration reloads its own chunk), so two chunks of each row are in flight.
  const XT* xr[kXbRows];
#pragma unroll
  for (int r = 0; r < kXbRows; ++r) xr[r] = X + min(row0 + r, n - 1) * ldx;
  int64_t c0 = (int64_t)lane * N;
  if (c0 < p_pad) {
    // two register sets used in turn: one chunk is summed while the next is loading (the last
    // chunk loads itself again, a valid address, in place of the chunk past the end)
    double b0[N], x0[kXbRows][N], b1[N], x1[kXbRows][N];
    auto load = [&](double (&bv)[N], double (&xv)[kXbRows][N], int64_t c) {
      load_dvec<N>(b + c, bv);
#pragma unroll
      for (int r = 0; r < kXbRows; ++r) XVec<XT>::load(xr[r] + c, xv[r]);
    };
    auto sum = [&](const double (&bv)[N], const double (&xv)[kXbRows][N]) {
#pragma unroll
      for (int r = 0; r < kXbRows; ++r) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) s = fma(xv[r][i], bv[i], s);
        acc[r] += s;
      }
    };
    load(b0, x0, c0);
    for (;;) {
      int64_t c1 = c0 + 64 * N;
      bool more = c1 < p_pad;
      load(b1, x1, more ? c1 : c0);
      __builtin_amdgcn_sched_barrier(0);
      sum(b0, x0);
      if (!more) break;
      c0 = c1;
      c1 = c0 + 64 * N;
      more = c1 < p_pad;
      load(b0, x0, more ? c1 : c0);
      __builtin_amdgcn_sched_barrier(0);
      sum(b1, x1);
      if (!more) break;
      c0 = c1;
    }
  }
  double lsum = 0.0;
#pragma unroll
  for (int r = 0; r < kXbRows; ++r) {
    const double v = wave_sum(acc[r]);
    const int64_t row = row0 + r;
    if (row < n) {
      if (lane == 0) u[row] = v;
      if (loss_part) lsum += loss_val(loss, v, y[row]);
    }
  }
  if (loss_part) {
    if (lane == 0) red[wid] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < kXbWaves; ++i) t += red[i];
      loss_part[blockIdx.x] = t;
    }
  }
}

// ------------------------------------------------------------------ h partials = X^T r

constexpr int kXtWaves = 4;
constexpr int kXtMaxChunk = 4096;

// part[chunk][j] = sum_{i in chunk} X_ij r_i over the workgroup's 64*N columns.
// mode 0 (solver): r_i = grad f_i(u_gamma_i), u_gamma = u^t + c (u^t - u^{t-1}) (ring slots
//   iter and iter-1), and column tile 0 also sums F*(-zeta) terms into fstar_part[chunk].
// mode 1 (plain product): r = u_base (an n-vector), no loss.
template <typename XT>
__global__ __launch_bounds__(256) void k_xt(const XT* __restrict__ X, int64_t ldx, int64_t n,
                                            int64_t p_pad, int64_t chunk_rows,
                                            const double* __restrict__ u_base, int64_t u_stride,
                                            const NodeDev* __restrict__ st,
                                            const double* __restrict__ y, int loss, int mode,
                                            double* __restrict__ part,
                                            double* __restrict__ fstar_part) {
  __shared__ double rs[kXtMaxChunk];
  __shared__ double red[kXtWaves * 64 * 8];
  if (st != nullptr && st->done) return;
  constexpr int N = XVec<XT>::N;
  const int tile = blockIdx.x;
  const int chunk = blockIdx.y;
  const int64_t r0 = (int64_t)chunk * chunk_rows;
  const int64_t r1 = min(n, r0 + chunk_rows);
  const int nr = (int)(r1 - r0);
  // residual vector for this chunk
  double fs = 0.0;
  if (mode == 0) {
    const int iter = st->iter;
    const double* ut = slot_ptr(u_base, u_stride, iter, 0);
    const double* utm = slot_ptr(u_base, u_stride, iter, 2);  // iter - 1 == iter + 2 (mod 3)
    const double c = st->c;
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {
      const int64_t row = r0 + i;
      const double ug = ut[row] + c * (ut[row] - utm[row]);
      rs[i] = loss_grad(loss, ug, y[row]);
      if (tile == 0) fs += fstar_term(loss, ug, y[row]);
    }
  } else {
    for (int i = threadIdx.x; i < nr; i += blockDim.x) rs[i] = u_base[r0 + i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t col = (int64_t)tile * 64 * N + (int64_t)lane * N;
  double acc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = 0.0;
  const XT* xp = X + r0 * ldx + col;
  int i = wid;
  // groups of four rows (one per wave stride); two register sets used in turn, so the next
  // group is loading while the current one is summed (a last group reloads itself, a valid
  // address, in place of the group past the end); the sum runs over the rows in order
  auto load4 = [&](double (&x)[4][N], int r) {
#pragma unroll
    for (int q = 0; q < 4; ++q) XVec<XT>::load(xp + (int64_t)(r + q * kXtWaves) * ldx, x[q]);
  };
  auto sum4 = [&](const double (&x)[4][N], int r) {
    const double a0 = rs[r], a1 = rs[r + kXtWaves], a2 = rs[r + 2 * kXtWaves],
                 a3 = rs[r + 3 * kXtWaves];
#pragma unroll
    for (int e = 0; e < N; ++e) {
      acc[e] = fma(x[0][e], a0, acc[e]);
      acc[e] = fma(x[1][e], a1, acc[e]);
      acc[e] = fma(x[2][e], a2, acc[e]);
      acc[e] = fma(x[3][e], a3, acc[e]);
    }
  };
  if (i + 3 * kXtWaves < nr) {
    double xa[4][N], xb[4][N];
    load4(xa, i);
    for (;;) {
      int nx = i + 4 * kXtWaves;
      bool more = nx + 3 * kXtWaves < nr;
      load4(xb, more ? nx : i);
      __builtin_amdgcn_sched_barrier(0);
      sum4(xa, i);
      i = nx;
      if (!more) break;
      nx = i + 4 * kXtWaves;
      more = nx + 3 * kXtWaves < nr;
      load4(xa, more ? nx : i);
      __builtin_amdgcn_sched_barrier(0);
      sum4(xb, i);
      i = nx;
      if (!more) break;
    }
  }
  for (; i < nr; i += kXtWaves) {
    double x0[N];
    XVec<XT>::load(xp + (int64_t)i * ldx, x0);
    const double a0 = rs[i];
#pragma unroll
    for (int e = 0; e < N; ++e) acc[e] = fma(x0[e], a0, acc[e]);
  }
  // reduce the four waves' partial column sums
#pragma unroll
  for (int e = 0; e < N; ++e) red[(wid * 64 + lane) * N + e] = acc[e];
  __syncthreads();
  for (int c = threadIdx.x; c < 64 * N; c += blockDim.x) {
    const int l = c / N, e = c % N;
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kXtWaves; ++w) s += red[(w * 64 + l) * N + e];
    part[(int64_t)chunk * p_pad + (int64_t)tile * 64 * N + c] = s;
  }
  if (mode == 0 && tile == 0) {
    __syncthreads();
    const double t = block_reduce(fs, red, OpAdd(), 0.0);
    if (threadIdx.x == 0) fstar_part[chunk] = t;
  }
}

// ------------------------------------------------------------------ gradient step

// h_j = sum_c part[c][j]; in solver mode also gamma = beta^t + c (beta^t - beta^{t-1}) and
// w = gamma - h / L. In plain mode (st == nullptr) only h is written.
__global__ __launch_bounds__(256) void k_grad_step(const double* __restrict__ part, int nchunks,
                                                   int64_t p_pad, const NodeDev* __restrict__ st,
                                                   const double* __restrict__ b_base,
                                                   int64_t b_stride, double inv_L, double shift,
                                                   double* __restrict__ h,
                                                   double* __restrict__ w,
                                                   double* __restrict__ gsq_part) {
  // with the eigen-perspective shift s the gradient is X^T grad f(X gamma) - 2 s gamma (App. D.2);
  // h receives the whole gradient, gsq_part the block's share of ||gamma||^2
  __shared__ double red[4];
  if (st != nullptr && st->done) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double gsq = 0.0;
  if (j < p_pad) {
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * p_pad + j];
    if (st != nullptr) {
      const int iter = st->iter;
      const double bt = slot_ptr(b_base, b_stride, iter, 0)[j];
      const double btm = slot_ptr(b_base, b_stride, iter, 2)[j];
      const double gamma = bt + st->c * (bt - btm);
      s -= 2.0 * shift * gamma;
      w[j] = gamma - s * inv_L;
      gsq = gamma * gamma;
    }
    h[j] = s;
  }
  if (gsq_part != nullptr) {
    gsq = block_reduce(gsq, red, OpAdd(), 0.0);
    if (threadIdx.x == 0) gsq_part[blockIdx.x] = gsq;
  }
}

// ------------------------------------------------------------------ prox

// One workgroup per node. w, h: p entries (node-major with stride ld for batches); cls: node
// class bytes; beta written to ring slot iter+1 of b_base (stride b_stride per node).
template <int E>
__global__ __launch_bounds__(1024) void k_prox(const double* __restrict__ w, int64_t w_ld,
                                               const double* __restrict__ h, int64_t h_ld,
                                               const uint8_t* __restrict__ cls_all,
                                               int64_t cls_ld, int64_t p, double rho, double M,
                                               double two_l2, NodeDev* __restrict__ st_all,
                                               double* __restrict__ b_base, int64_t b_stride,
                                               int64_t b_node_stride, int want_bsq) {
  __shared__ ProxSmem sm;
  const int node = blockIdx.x;
  NodeDev* st = st_all + node;
  if (st->done) return;
  const int iter = st->iter;
  const double* wn = w + (int64_t)node * w_ld;
  const uint8_t* cls_n = cls_all + (int64_t)node * cls_ld;
  __shared__ double vbuf[ProxVals<E>::nl * kProxThreads];
  ProxVals<E> pv;
  pv.sl = vbuf;
  uint64_t cb = 0;
  uint32_t neg = 0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
    double w = 0.0;
    int cs = CLS_PAD;
    if (j < p) { w = wn[j]; cs = cls_n[j]; }
    neg |= (w < 0.0 ? 1u : 0u) << s;
    pv.set(s, rho * fabs(w));
    cb |= (uint64_t)cs << (2 * s);
  }
  double* bout = slot_ptr(b_base + (int64_t)node * b_node_stride, b_stride, iter, 1);
  double bsq = 0.0;
  const ProxOut po = node_prox<E>(
      [&](int s) { return pv.get(s); }, neg, cb, st->kp, st->nfree, rho, M, st->vstar,
      [&](int s, double b) {
        const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
        if (j < p) bout[j] = b;
        bsq += b * b;
      },
      sm);
  if (want_bsq) bsq = bsum(bsq, sm);
  const bool check = ((iter % st->check_every) == 0) || (iter >= st->max_iter);
  double gs = 0.0;
  if (check && h != nullptr) {
    const double* hn = h + (int64_t)node * h_ld;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
      pv.set(s, (j < p) ? fabs(hn[j]) : 0.0);
    }
    gs = gstar_node<E>([&](int s) { return pv.get(s); }, two_l2, cb, st->kp, st->nfree, M, sm);
  }
  if (threadIdx.x == 0) {
    st->g_new = po.gval;
    st->gstar_new = gs;
    st->bsq_new = bsq;
    st->checked = check ? 1 : 0;
    st->vstar = po.vstar;
  }
}

// ------------------------------------------------------------------ finish an iteration

// One workgroup (256 threads) per node. Sums the loss partials of k_xb and the F* partials of
// k_xt, forms L^{t+1} = f(X beta^{t+1}) + 2 lambda2 g_node(beta^{t+1}), applies the value
// restart of Alg. 3, keeps the best primal point, forms the weak-duality bound
// D = -F*(-zeta) - 2 lambda2 g_node*(X^T zeta / (2 lambda2)) with zeta = -grad f(X gamma^t)
// (X^T zeta = -h), and applies the stopping rules.
__global__ __launch_bounds__(256) void k_finish(const double* __restrict__ loss_part,
                                                int nloss, const double* __restrict__ fstar_part,
                                                int nfstar, double two_l2,
                                                NodeDev* __restrict__ st,
                                                const double* __restrict__ b_base,
                                                int64_t b_stride, double* __restrict__ b_best,
                                                int64_t p, double shift,
                                                const double* __restrict__ gsq_part, int ngsq) {
  __shared__ double red[4];
  __shared__ int improve;
  if (st->done) return;
  double a = 0.0, f = 0.0, gsq = 0.0;
  for (int i = threadIdx.x; i < nloss; i += blockDim.x) a += loss_part[i];
  for (int i = threadIdx.x; i < nfstar; i += blockDim.x) f += fstar_part[i];
  if (gsq_part != nullptr)
    for (int i = threadIdx.x; i < ngsq; i += blockDim.x) gsq += gsq_part[i];
  a = block_reduce(a, red, OpAdd(), 0.0);
  f = block_reduce(f, red, OpAdd(), 0.0);
  gsq = block_reduce(gsq, red, OpAdd(), 0.0);
  const int iter = st->iter;
  if (threadIdx.x == 0) {
    // eigen-perspective shift s (App. D.2): objective f - s ||beta||^2 + 2 lambda_eig g, and the
    // bound gains s ||gamma||^2 (two_l2 is then 2 lambda_eig); s = 0 is the plain relaxation
    const double Lnew = a - shift * st->bsq_new + two_l2 * st->g_new;
    st->L_work = Lnew;
    if (Lnew >= st->L_prev) { st->phi = 1.0; st->restarts += 1; }
    else st->phi += 1.0;
    st->L_prev = Lnew;
    improve = 0;
    if (Lnew < st->P_best) { st->P_best = Lnew; st->best_iter = iter + 1; improve = 1; }
    if (st->checked) {
      const double D = -f - two_l2 * st->gstar_new + shift * gsq;
      if (D > st->D_best) st->D_best = D;
    }
    const double gap = (st->P_best - st->D_best) / fmax(fabs(st->P_best), 1.0);
    int status = kRunning;
    if (!isfinite(Lnew) && !isinf(Lnew)) status = 3;           // NUMERIC (NaN)
    else if (gap <= st->tol) status = 0;                      // CONVERGED
    else if (isfinite(st->incumbent) && st->D_best > st->incumbent) status = 5;  // PRUNED
    else if (isfinite(st->incumbent) && st->P_best < st->incumbent) status = 6;  // BELOW_INC.
    else if (iter + 1 > st->max_iter) status = 1;             // NOT_CONVERGED
    st->iter = iter + 1;
    st->c = st->phi / (st->phi + 3.0);
    if (status != kRunning) { st->status = status; st->done = 1; }
  }
  __syncthreads();
  if (improve) {
    const double* bn = slot_ptr(b_base, b_stride, iter, 1);
    for (int64_t j = threadIdx.x; j < p; j += blockDim.x) b_best[j] = bn[j];
  }
}

// Initial state after u^1 = X beta^1 has been formed with loss partials.
__global__ void k_init_state(const double* __restrict__ loss_part, int nloss, double L0_g,
                             NodeDev* __restrict__ st) {
  __shared__ double red[4];
  double a = 0.0;
  for (int i = threadIdx.x; i < nloss; i += blockDim.x) a += loss_part[i];
  a = block_reduce(a, red, OpAdd(), 0.0);
  if (threadIdx.x == 0) {
    st->L_prev = a + L0_g;  // L0_g = 2 lambda2 g(beta^1), +inf when unknown (warm start)
    st->P_best = st->L_prev;
    st->L_work = st->L_prev;
  }
}

// ------------------------------------------------------------------ launch wrappers

static int xt_chunks(int64_t n, int64_t ntiles, int64_t* rows) {
  int64_t nch = std::max<int64_t>(1, 1024 / std::max<int64_t>(1, ntiles));
  nch = std::max<int64_t>(nch, (n + kXtMaxChunk - 1) / kXtMaxChunk);
  nch = std::min<int64_t>(nch, std::max<int64_t>(1, (n + 63) / 64));
  int64_t cr = (n + nch - 1) / nch;
  nch = (n + cr - 1) / cr;
  *rows = cr;
  return (int)nch;
}

int64_t xt_vec(int xtype) { return xtype == XT_F64 ? 2 : (xtype == XT_F32 ? 4 : 8); }

PlainGeom plain_geometry(int xtype, int64_t n, int64_t p_pad) {
  PlainGeom g;
  const int64_t N = xt_vec(xtype);
  g.ntiles = p_pad / (64 * N);
  g.nchunks = xt_chunks(n, g.ntiles, &g.chunk_rows);
  g.nxb = (int)((n + kXbRows * kXbWaves - 1) / (kXbRows * kXbWaves));
  return g;
}

template <typename XT>
static void launch_xb_t(const void* X, int64_t ldx, int64_t n, int64_t p_pad, const double* b,
                        int64_t bs, double* u, int64_t us, const NodeDev* st, const double* y,
                        int loss, double* loss_part, hipStream_t stream) {
  const int nb = (int)((n + kXbRows * kXbWaves - 1) / (kXbRows * kXbWaves));
  hipLaunchKernelGGL(k_xb<XT>, dim3(nb), dim3(256), 0, stream, (const XT*)X, ldx, n, p_pad, b,
                     bs, u, us, st, y, loss, loss_part);
}

void launch_xb(int xtype, const void* X, int64_t ldx, int64_t n, int64_t p_pad, const double* b,
               int64_t bs, double* u, int64_t us, const NodeDev* st, const double* y, int loss,
               double* loss_part, hipStream_t stream) {
  if (xtype == XT_F64) launch_xb_t<double>(X, ldx, n, p_pad, b, bs, u, us, st, y, loss, loss_part, stream);
  else if (xtype == XT_F32) launch_xb_t<float>(X, ldx, n, p_pad, b, bs, u, us, st, y, loss, loss_part, stream);
  else launch_xb_t<uint16_t>(X, ldx, n, p_pad, b, bs, u, us, st, y, loss, loss_part, stream);
}

template <typename XT>
static void launch_xt_t(const void* X, int64_t ldx, int64_t n, int64_t p_pad,
                        const PlainGeom& g, const double* u, int64_t us, const NodeDev* st,
                        const double* y, int loss, int mode, double* part, double* fpart,
                        hipStream_t stream) {
  hipLaunchKernelGGL(k_xt<XT>, dim3((unsigned)g.ntiles, (unsigned)g.nchunks), dim3(256), 0,
                     stream, (const XT*)X, ldx, n, p_pad, g.chunk_rows, u, us, st, y, loss, mode,
                     part, fpart);
}

void launch_xt(int xtype, const void* X, int64_t ldx, int64_t n, int64_t p_pad,
               const PlainGeom& g, const double* u, int64_t us, const NodeDev* st,
               const double* y, int loss, int mode, double* part, double* fpart,
               hipStream_t stream) {
  if (xtype == XT_F64) launch_xt_t<double>(X, ldx, n, p_pad, g, u, us, st, y, loss, mode, part, fpart, stream);
  else if (xtype == XT_F32) launch_xt_t<float>(X, ldx, n, p_pad, g, u, us, st, y, loss, mode, part, fpart, stream);
  else launch_xt_t<uint16_t>(X, ldx, n, p_pad, g, u, us, st, y, loss, mode, part, fpart, stream);
}

void launch_grad_step(const double* part, int nchunks, int64_t p_pad, const NodeDev* st,
                      const double* b_base, int64_t b_stride, double inv_L, double* h, double* w,
                      hipStream_t stream, double shift, double* gsq_part) {
  hipLaunchKernelGGL(k_grad_step, dim3((unsigned)((p_pad + 255) / 256)), dim3(256), 0, stream,
                     part, nchunks, p_pad, st, b_base, b_stride, inv_L, shift, h, w, gsq_part);
}

int prox_elems(int64_t p) {
  // elements per thread: powers of two and the steps of 1.5 between the larger ones, so that at
  // most a third of a thread's element slots go unused for p above 4096 (and 10 and 20, which fit
  // p = 10000 and p = 20000 with 2% of the slots unused)
  const int64_t e = (p + kProxThreads - 1) / kProxThreads;
  for (int c : {1, 2, 4, 6, 8, 10, 12, 16, 20, 24, 32})
    if (e <= c) return c;
  return -1;
}

void launch_prox(int nodes, const double* w, int64_t w_ld, const double* h, int64_t h_ld,
                 const uint8_t* cls, int64_t cls_ld, int64_t p, double rho, double M,
                 double two_l2, NodeDev* st, double* b_base, int64_t b_stride,
                 int64_t b_node_stride, hipStream_t stream, int want_bsq) {
  const int E = prox_elems(p);
#define CGL_PROX_CASE(EE)                                                                       \
  case EE:                                                                                      \
    hipLaunchKernelGGL(k_prox<EE>, dim3(nodes), dim3(kProxThreads), 0, stream, w, w_ld, h, h_ld, \
                       cls, cls_ld, p, rho, M, two_l2, st, b_base, b_stride, b_node_stride,     \
                       want_bsq);                                                               \
    break;
  switch (E) {
    CGL_PROX_CASE(1)
    CGL_PROX_CASE(2)
    CGL_PROX_CASE(4)
    CGL_PROX_CASE(6)
    CGL_PROX_CASE(8)
    CGL_PROX_CASE(10)
    CGL_PROX_CASE(12)
    CGL_PROX_CASE(16)
    CGL_PROX_CASE(20)
    CGL_PROX_CASE(24)
    CGL_PROX_CASE(32)
    default:
      break;
  }
#undef CGL_PROX_CASE
}

void launch_finish(const double* loss_part, int nloss, const double* fstar_part, int nfstar,
                   double two_l2, NodeDev* st, const double* b_base, int64_t b_stride,
                   double* b_best, int64_t p, hipStream_t stream, double shift,
                   const double* gsq_part, int ngsq) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, stream, loss_part, nloss, fstar_part,
                     nfstar, two_l2, st, b_base, b_stride, b_best, p, shift, gsq_part, ngsq);
}

void launch_init_state(const double* loss_part, int nloss, double L0_g, NodeDev* st,
                       hipStream_t stream) {
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(256), 0, stream, loss_part, nloss, L0_g, st);
}

// ------------------------------------------------------------------ power iteration step

// z holds X^T X v for a unit v: lam = v . z (Rayleigh quotient), then v = z / ||z||.
__global__ __launch_bounds__(1024) void k_power_normalize(const double* __restrict__ z,
                                                          double* __restrict__ v, int64_t p,
                                                          double* __restrict__ lam) {
  __shared__ double red[16];
  double nz = 0.0, vz = 0.0;
  for (int64_t j = threadIdx.x; j < p; j += blockDim.x) {
    nz += z[j] * z[j];
    vz += v[j] * z[j];
  }
  nz = block_reduce(nz, red, OpAdd(), 0.0);
  vz = block_reduce(vz, red, OpAdd(), 0.0);
  const double inv = nz > 0.0 ? 1.0 / sqrt(nz) : 0.0;
  for (int64_t j = threadIdx.x; j < p; j += blockDim.x) v[j] = z[j] * inv;
  if (threadIdx.x == 0) *lam = vz;
}

void launch_power_normalize(const double* z, double* v, int64_t p, double* lam,
                            hipStream_t stream) {
  hipLaunchKernelGGL(k_power_normalize, dim3(1), dim3(1024), 0, stream, z, v, p, lam);
}

// ------------------------------------------------------------------ certification pieces

// r_i = grad f_i(u_i) and F*(-zeta) partial sums with zeta = -r (mode 2 of the X^T pass is a
// plain product of X^T with this r).
__global__ __launch_bounds__(256) void k_resid(const double* __restrict__ u,
                                               const double* __restrict__ y, int64_t n, int loss,
                                               double* __restrict__ r,
                                               double* __restrict__ part2) {
  __shared__ double red[8];
  double lsum = 0.0, fsum = 0.0;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    r[i] = loss_grad(loss, u[i], y[i]);
    lsum = loss_val(loss, u[i], y[i]);
    fsum = fstar_term(loss, u[i], y[i]);
  }
  lsum = block_reduce(lsum, red, OpAdd(), 0.0);
  fsum = block_reduce(fsum, red, OpAdd(), 0.0);
  if (threadIdx.x == 0) {
    part2[2 * blockIdx.x] = lsum;
    part2[2 * blockIdx.x + 1] = fsum;
  }
}

void launch_resid(const double* u, const double* y, int64_t n, int loss, double* r,
                  double* part2, hipStream_t stream) {
  hipLaunchKernelGGL(k_resid, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, u, y, n,
                     loss, r, part2);
}

// One workgroup per node: out[2 node] = g_node(beta) (Alg. 2; +inf outside the domain) and
// out[2 node + 1] = g_node*(-h / (2 lambda2)) (Lemma 2).
template <int E>
__global__ __launch_bounds__(1024) void k_g_gstar(const double* __restrict__ beta, int64_t b_ld,
                                                  const double* __restrict__ h, int64_t h_ld,
                                                  const uint8_t* __restrict__ cls_all,
                                                  int64_t cls_ld, const NodeDev* __restrict__ st_all,
                                                  int64_t p, double M, double two_l2,
                                                  double* __restrict__ out) {
  __shared__ ProxSmem sm;
  const int node = blockIdx.x;
  const NodeDev* st = st_all + node;
  const int kp = st->kp, nfree = st->nfree;
  const uint8_t* cl = cls_all + (int64_t)node * cls_ld;
  // |beta| first (Alg. 2), then |h| (the conjugate) in the per-thread value slice
  __shared__ double vbuf[ProxVals<E>::nl * kProxThreads];
  ProxVals<E> pv;
  pv.sl = vbuf;
  uint64_t cb = 0;
  uint32_t fm = 0;
  double absF = 0.0, sq1 = 0.0, mx = 0.0;
  int bad = 0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
    int c = CLS_PAD;
    double bj = 0.0;
    if (j < p) {
      bj = beta[(int64_t)node * b_ld + j];
      c = cl[j];
    }
    pv.set(s, fabs(bj));
    cb |= (uint64_t)c << (2 * s);
    if (c == CLS_FREE) fm |= 1u << s;
    if (c == CLS_ZERO && bj != 0.0) bad = 1;
    if (c == CLS_ONE) { sq1 += bj * bj; if (fabs(bj) > M * (1.0 + 1e-12)) bad = 1; }
    if (c == CLS_FREE) { absF += fabs(bj); mx = fmax(mx, fabs(bj)); }
  }
  absF = bsum(absF, sm);
  sq1 = bsum(sq1, sm);
  mx = bmax(mx, sm);
  bad = bsum_i(bad, sm);
  double g = 0.0;
  if (bad || mx > M * (1.0 + 1e-12) || absF > (double)kp * M * (1.0 + 1e-12) ||
      (kp <= 0 && absF > 0.0)) {
    g = HUGE_VAL;
  } else if (kp > 0 && nfree > 0) {
    if (kp >= nfree) {
      double sq = 0.0;
#pragma unroll
      for (int s = 0; s < E; ++s) if ((fm >> s) & 1u) sq += pv.get(s) * pv.get(s);
      g = 0.5 * bsum(sq, sm);
    } else {
      // top-kp magnitudes of beta_F, sorted decreasingly, then Alg. 2
      auto K = [&](int s) { return dbits(pv.get(s)); };
      const Select sel = radix_select_desc<E>(K, fm, kp, sm);
      if (threadIdx.x == 0) { sm.head_fill = 0; sm.ties_left = sel.exact ? sel.take : 0; }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < E; ++s) {
        if (!((fm >> s) & 1u)) continue;
        const uint64_t ks = K(s);
        bool hsel = !sel.exact ? ks >= sel.lo
                               : (ks > sel.lo || (ks == sel.lo &&
                                                  atomicSub(&sm.ties_left, 1) > 0));
        if (hsel) sm.hu[atomicAdd(&sm.head_fill, 1)] = pv.get(s);
      }
      __syncthreads();
      sort_head_desc(kp, sm);
      if (threadIdx.x == 0) sm.b_dbl[3] = alg2_from_sorted(sm.hu, kp, kp, absF);
      __syncthreads();
      g = sm.b_dbl[3];
    }
  }
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int64_t j = (int64_t)s * kProxThreads + threadIdx.x;
    pv.set(s, (j < p) ? fabs(h[(int64_t)node * h_ld + j]) : 0.0);
  }
  const double gn = 0.5 * sq1 + g;
  const double gs = gstar_node<E>([&](int s) { return pv.get(s); }, two_l2, cb, kp, nfree, M, sm);
  if (threadIdx.x == 0) {
    out[2 * node] = gn;
    out[2 * node + 1] = gs;
  }
}

void launch_g_gstar(int nodes, const double* beta, int64_t b_ld, const double* h, int64_t h_ld,
                    const uint8_t* cls, int64_t cls_ld, const NodeDev* st, int64_t p, double M,
                    double two_l2, double* out, hipStream_t stream) {
  const int E = prox_elems(p);
#define CGL_G_CASE(EE)                                                                         \
  case EE:                                                                                     \
    hipLaunchKernelGGL(k_g_gstar<EE>, dim3(nodes), dim3(kProxThreads), 0, stream, beta, b_ld, h, \
                       h_ld, cls, cls_ld, st, p, M, two_l2, out);                              \
    break;
  switch (E) {
    CGL_G_CASE(1)
    CGL_G_CASE(2)
    CGL_G_CASE(4)
    CGL_G_CASE(6)
    CGL_G_CASE(8)
    CGL_G_CASE(10)
    CGL_G_CASE(12)
    CGL_G_CASE(16)
    CGL_G_CASE(20)
    CGL_G_CASE(24)
    CGL_G_CASE(32)
    default:
      break;
  }
#undef CGL_G_CASE
}

// =====================================================================================
// Count of non-finite entries of a stored design (any precision; padding is zero). The counter
// starts at zero; each workgroup adds its count once.
// =====================================================================================
template <typename XT>
__device__ __forceinline__ bool not_finite(XT v);
template <>
__device__ __forceinline__ bool not_finite<double>(double v) { return !isfinite(v); }
template <>
__device__ __forceinline__ bool not_finite<float>(float v) { return !isfinite(v); }
template <>
__device__ __forceinline__ bool not_finite<uint16_t>(uint16_t v) { return (v & 0x7f80u) == 0x7f80u; }

template <typename XT>
__global__ __launch_bounds__(256) void k_count_nonfinite(const XT* __restrict__ X, int64_t count,
                                                         int* bad) {
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256)
    c += not_finite<XT>(X[i]) ? 1 : 0;
  if (c) atomicAdd(&sbad, c);
  __syncthreads();
  if (threadIdx.x == 0 && sbad) atomicAdd(bad, sbad);
}

void launch_count_nonfinite(int xtype, const void* X, int64_t count, int* bad, hipStream_t s) {
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (count + 255) / 256));
  if (xtype == XT_F64)
    hipLaunchKernelGGL(k_count_nonfinite<double>, dim3(grid), dim3(256), 0, s,
                       (const double*)X, count, bad);
  else if (xtype == XT_F32)
    hipLaunchKernelGGL(k_count_nonfinite<float>, dim3(grid), dim3(256), 0, s, (const float*)X,
                       count, bad);
  else
    hipLaunchKernelGGL(k_count_nonfinite<uint16_t>, dim3(grid), dim3(256), 0, s,
                       (const uint16_t*)X, count, bad);
}


// Count of differing 32-bit words of two device buffers (words < count); the counter starts at
// zero; each workgroup adds its count once.
__global__ __launch_bounds__(256) void k_count_diff(const uint32_t* __restrict__ a,
                                                    const uint32_t* __restrict__ b, int64_t count,
                                                    int* diff) {
  __shared__ int sd;
  if (threadIdx.x == 0) sd = 0;
  __syncthreads();
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256)
    c += a[i] != b[i] ? 1 : 0;
  if (c) atomicAdd(&sd, c);
  __syncthreads();
  if (threadIdx.x == 0 && sd) atomicAdd(diff, sd);
}

void launch_count_diff(const void* a, const void* b, int64_t words, int* diff, hipStream_t s) {
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (words + 255) / 256));
  hipLaunchKernelGGL(k_count_diff, dim3(grid), dim3(256), 0, s, (const uint32_t*)a,
                     (const uint32_t*)b, words, diff);
}

}  // namespace cgl

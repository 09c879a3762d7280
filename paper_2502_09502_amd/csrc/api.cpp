// C-ABI of libcertglm: contexts, problems, the plain FP64 per-node solve and the certification
// utilities. The batched mixed-precision engine and the server live in batch.cpp / server.cpp.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/certglm.h"
#include "batch.h"
#include "engine.h"
#include "kernels.h"
#include "losses.h"
#include "prox.h"

// Timing events: read only after the stream has been synchronised, so they need no system-scope
// fence (which would write back caches at every record and delay the next kernel).
hipEvent_t cgl_ctx::event(size_t i) {
  while (events.size() <= i) {
    hipEvent_t e;
    CGL_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    events.push_back(e);
  }
  return events[i];
}

// Tuning cache: one line per choice, "<arch> <pass> <M> <K> <nodes> <split>". CGL_TUNE_CACHE
// names the file ("0" or an empty value: no file); otherwise $XDG_CACHE_HOME/certglm/splits.txt
// or $HOME/.cache/certglm/splits.txt. A file that cannot be read or written is ignored.
static std::string tune_cache_path() {
  const char* e = std::getenv("CGL_TUNE_CACHE");
  if (e) return (e[0] == '\0' || (e[0] == '0' && e[1] == '\0')) ? std::string() : std::string(e);
  if (const char* x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/certglm/splits.txt";
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/certglm/splits.txt";
  return std::string();
}

void cgl_ctx::load_tuning() {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char a[64];
  long long pass, m, k, nodes;
  int ks;
  while (std::fscanf(f, "%63s %lld %lld %lld %lld %d", a, &pass, &m, &k, &nodes, &ks) == 6)
    if (arch == a && ks >= 1) tuned_split[{pass, m, k, nodes}] = ks;
  std::fclose(f);
}

void cgl_ctx::save_tuning(const std::array<int64_t, 4>& key, int choice) const {
  const std::string path = tune_cache_path();
  if (path.empty() || arch.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    // create the directory chain (one level per component; errors are ignored)
    for (size_t q = path.find('/', 1); q != std::string::npos && q <= slash; q = path.find('/', q + 1))
      (void)mkdir(path.substr(0, q).c_str(), 0755);
  }
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s %lld %lld %lld %lld %d\n", arch.c_str(), (long long)key[0],
               (long long)key[1], (long long)key[2], (long long)key[3], choice);
  std::fclose(f);
}

cgl_ctx::~cgl_ctx() {
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

namespace cgl {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

[[noreturn]] void invalid(const std::string& m) { throw InvalidArg{m}; }

DevBuf::~DevBuf() { reset(); }
void DevBuf::reset() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}
void DevBuf::alloc(size_t b) {
  if (b <= bytes && ptr) return;
  reset();
  if (b == 0) b = 8;
  if (hipMalloc(&ptr, b) != hipSuccess) {
    ptr = nullptr;
    throw std::bad_alloc();
  }
  bytes = b;
}

int64_t pad_cols(int64_t p) { return (p + 511) / 512 * 512; }

// Longest vector of the standalone prox (cgl_prox_node_batch); problems stop at 32768.
constexpr int64_t kProxMaxP = 1 << 20;
// Longest vector the standalone prox holds per thread (16 values in LDS slices).
constexpr int64_t kProxHeldP = 16 * 1024;

// ------------------------------------------------------------------ node validation

NodeHost make_node_host(const cgl_node& nd, int64_t p, int k) {
  NodeHost h;
  h.cls.assign((size_t)p, CLS_FREE);
  if (nd.n_zero < 0 || nd.n_in < 0) invalid("negative fixed-set size");
  if ((nd.n_zero > 0 && !nd.fixed_zero) || (nd.n_in > 0 && !nd.fixed_in))
    invalid("fixed-set pointer is NULL");
  for (int32_t i = 0; i < nd.n_zero; ++i) {
    const int32_t j = nd.fixed_zero[i];
    if (j < 0 || j >= p) invalid("fixed_zero index out of range");
    if (h.cls[(size_t)j] != CLS_FREE) invalid("duplicate fixed_zero index");
    h.cls[(size_t)j] = CLS_ZERO;
  }
  for (int32_t i = 0; i < nd.n_in; ++i) {
    const int32_t j = nd.fixed_in[i];
    if (j < 0 || j >= p) invalid("fixed_in index out of range");
    if (h.cls[(size_t)j] == CLS_ZERO) invalid("index fixed both to zero and to one");
    if (h.cls[(size_t)j] == CLS_ONE) invalid("duplicate fixed_in index");
    h.cls[(size_t)j] = CLS_ONE;
  }
  if (!(nd.tol >= 0.0)) invalid("tol must be >= 0");
  if (nd.max_iter < 1) invalid("max_iter must be >= 1");
  if (nd.check_every < 1) invalid("check_every must be >= 1");
  if (nd.precision != CGL_PREC_F64 && nd.precision != CGL_PREC_MIXED) invalid("bad precision");
  if (std::isnan(nd.incumbent)) invalid("incumbent is NaN");
  h.kp = k - nd.n_in;
  h.nfree = (int)(p - nd.n_zero - nd.n_in);
  h.infeasible = h.kp < 0;
  if (h.kp > kMaxHead && h.kp < h.nfree)
    invalid("k - |Z1| > 256 with more free coordinates than that is not supported");
  if (nd.warm_start) {
    for (int64_t j = 0; j < p; ++j)
      if (!std::isfinite(nd.warm_start[j])) invalid("non-finite warm start");
  }
  return h;
}

NodeDev make_node_dev(const cgl_node& nd, const NodeHost& h) {
  NodeDev s;
  std::memset(&s, 0, sizeof(s));
  s.phi = 1.0;
  s.c = 0.25;
  s.L_prev = HUGE_VAL;
  s.P_best = HUGE_VAL;
  s.D_best = -HUGE_VAL;
  s.iter = 1;
  s.status = kRunning;
  s.kp = h.kp;
  s.nfree = h.nfree;
  s.max_iter = nd.max_iter;
  s.check_every = nd.check_every;
  s.tol = nd.tol;
  s.incumbent = nd.incumbent;
  return s;
}

void fill_result(const NodeDev& s, cgl_result* r) {
  r->primal = s.P_best;
  r->lower_bound = s.D_best;
  r->gap_abs = s.P_best - s.D_best;
  r->gap_rel = r->gap_abs / std::max(std::fabs(s.P_best), 1.0);
  r->iters = s.iter - 1;
  r->restarts = s.restarts;
  r->status = s.status == kRunning ? CGL_NOT_CONVERGED : s.status;
  r->recentres = s.recentres;
  r->err_vs_fp64_est = 0.0;
}

void infeasible_result(cgl_result* r, double* beta_out, int64_t p) {
  r->primal = HUGE_VAL;
  r->lower_bound = HUGE_VAL;
  r->gap_abs = 0.0;
  r->gap_rel = 0.0;
  r->iters = 0;
  r->restarts = 0;
  r->status = CGL_INFEASIBLE;
  r->recentres = 0;
  r->err_vs_fp64_est = 0.0;
  if (beta_out) std::fill(beta_out, beta_out + p, 0.0);
}

// ------------------------------------------------------------------ problem setup

// Non-finite entries of a host X (n x p, leading dimension ldx): NaN or infinity; for BF16 the
// exponent bits all set.
static int64_t count_nonfinite_host(const void* X, int32_t x_dtype, int64_t n, int64_t p,
                                    int64_t ldx) {
  int64_t bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (x_dtype == CGL_F64) {
      const double* r = static_cast<const double*>(X) + i * ldx;
      for (int64_t j = 0; j < p; ++j) bad += std::isfinite(r[j]) ? 0 : 1;
    } else if (x_dtype == CGL_F32) {
      const float* r = static_cast<const float*>(X) + i * ldx;
      for (int64_t j = 0; j < p; ++j) bad += std::isfinite(r[j]) ? 0 : 1;
    } else {
      const uint16_t* r = static_cast<const uint16_t*>(X) + i * ldx;
      for (int64_t j = 0; j < p; ++j) bad += (r[j] & 0x7f80u) == 0x7f80u ? 1 : 0;
    }
  }
  return bad;
}

static void upload_X(Problem& P, const void* X, int32_t x_mem, int64_t ldx) {
  const size_t es = P.xtype == XT_F64 ? 8 : (P.xtype == XT_F32 ? 4 : 2);
  P.X.alloc((size_t)P.n * P.ldx * es);
  hipStream_t s = P.ctx->stream;
  CGL_HIP(hipMemsetAsync(P.X.ptr, 0, (size_t)P.n * P.ldx * es, s));
  const hipMemcpyKind kind = x_mem == CGL_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  CGL_HIP(hipMemcpy2DAsync(P.X.ptr, (size_t)P.ldx * es, X, (size_t)ldx * es, (size_t)P.p * es,
                           (size_t)P.n, kind, s));
  CGL_HIP(hipStreamSynchronize(s));
}

static double power_lambda_max(Problem& P) {
  hipStream_t s = P.ctx->stream;
  const PlainGeom g = plain_geometry(P.xtype, P.n, P.ldx);
  DevBuf v, u, part, z, lam;
  v.alloc(P.ldx * 8);
  u.alloc(P.n * 8);
  part.alloc((size_t)g.nchunks * P.ldx * 8);
  z.alloc(P.ldx * 8);
  lam.alloc(8);
  // deterministic start: v_j = 1 + (j mod 7) / 10, normalised on the device
  std::vector<double> v0((size_t)P.ldx, 0.0);
  for (int64_t j = 0; j < P.p; ++j) v0[(size_t)j] = 1.0 + (double)(j % 7) / 10.0;
  CGL_HIP(hipMemcpyAsync(v.ptr, v0.data(), P.ldx * 8, hipMemcpyHostToDevice, s));
  launch_power_normalize(v.as<double>(), v.as<double>(), P.ldx, lam.as<double>(), s);
  double prev = 0.0, cur = 0.0;
  for (int it = 1; it <= 2000; ++it) {
    launch_xb(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, v.as<double>(), 0, u.as<double>(), 0, nullptr,
              nullptr, 0, nullptr, s);
    launch_xt(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, g, u.as<double>(), 0, nullptr, nullptr, 0, 1,
              part.as<double>(), nullptr, s);
    launch_grad_step(part.as<double>(), g.nchunks, P.ldx, nullptr, nullptr, 0, 0.0,
                     z.as<double>(), nullptr, s);
    launch_power_normalize(z.as<double>(), v.as<double>(), P.ldx, lam.as<double>(), s);
    if (it % 20 == 0) {
      CGL_HIP(hipMemcpyAsync(&cur, lam.ptr, 8, hipMemcpyDeviceToHost, s));
      CGL_HIP(hipStreamSynchronize(s));
      if (it >= 40 && std::fabs(cur - prev) <= 1e-9 * std::fabs(cur)) break;
      prev = cur;
    }
  }
  CGL_HIP(hipMemcpyAsync(&cur, lam.ptr, 8, hipMemcpyDeviceToHost, s));
  CGL_HIP(hipStreamSynchronize(s));
  return cur;
}

// ------------------------------------------------------------------ plain solve

void PlainWork::ensure(Problem& P) {
  if (ready) return;
  geom = plain_geometry(P.xtype, P.n, P.ldx);
  bring.alloc(3 * P.ldx * 8);
  uring.alloc(3 * P.n * 8);
  bbest.alloc(P.ldx * 8);
  w.alloc(P.ldx * 8);
  h.alloc(P.ldx * 8);
  part.alloc((size_t)geom.nchunks * P.ldx * 8);
  fpart.alloc((size_t)geom.nchunks * 8);
  lpart.alloc((size_t)geom.nxb * 8);
  cls.alloc(P.ldx);
  st.alloc(sizeof(NodeDev));
  gsq.alloc((size_t)((P.ldx + 255) / 256) * 8);
  CGL_HIP(hipHostMalloc(&st_host, sizeof(NodeDev), hipHostMallocDefault));
  CGL_HIP(hipEventCreateWithFlags(&chunk_ev, hipEventDisableTiming));
  ready = true;
}

PlainWork::~PlainWork() {
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (st_host) (void)hipHostFree(st_host);
  if (chunk_ev) (void)hipEventDestroy(chunk_ev);
}

// One iteration of Alg. 3 on the plain path. ev (optional): four events bracketing the X^T pass
// and the X pass, for kernel timing.
static void plain_iteration(Problem& P, PlainWork& W, hipStream_t s, hipEvent_t* ev = nullptr) {
  const double two_l2 = 2.0 * (P.lam2 + P.shift);  // 2 lambda_eig with the eigen shift
  const bool eig = P.shift != 0.0;
  const int ngsq = (int)((P.ldx + 255) / 256);
  NodeDev* st = W.st.as<NodeDev>();
  if (ev) CGL_HIP(hipEventRecord(ev[0], s));
  launch_xt(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, W.geom, W.uring.as<double>(), P.n, st,
            P.y.as<double>(), P.loss, 0, W.part.as<double>(), W.fpart.as<double>(), s);
  if (ev) CGL_HIP(hipEventRecord(ev[1], s));
  launch_grad_step(W.part.as<double>(), W.geom.nchunks, P.ldx, st, W.bring.as<double>(), P.ldx,
                   1.0 / P.L, W.h.as<double>(), W.w.as<double>(), s, P.shift,
                   eig ? W.gsq.as<double>() : nullptr);
  launch_prox(1, W.w.as<double>(), 0, W.h.as<double>(), 0, W.cls.as<uint8_t>(), 0, P.p, P.rho,
              P.M, two_l2, st, W.bring.as<double>(), P.ldx, 0, s, eig ? 1 : 0);
  if (ev) CGL_HIP(hipEventRecord(ev[2], s));
  launch_xb(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, W.bring.as<double>(), P.ldx,
            W.uring.as<double>(), P.n, st, P.y.as<double>(), P.loss, W.lpart.as<double>(), s);
  if (ev) CGL_HIP(hipEventRecord(ev[3], s));
  launch_finish(W.lpart.as<double>(), W.geom.nxb, W.fpart.as<double>(), W.geom.nchunks, two_l2,
                st, W.bring.as<double>(), P.ldx, W.bbest.as<double>(), P.p, s, P.shift,
                eig ? W.gsq.as<double>() : nullptr, ngsq);
}

static bool use_graphs() {
  const char* e = std::getenv("CGL_NO_GRAPH");
  return !(e && e[0] == '1');
}

// The plain solve in steps, so that a caller (the server) can advance it between other work:
// plain_begin sets the node up and queues its first objective, plain_launch queues a chunk of
// iterations with the copy of the state to the host and the chunk event, plain_after_chunk (once
// the event has completed) books the kernel timing and says whether the node is finished, and
// plain_end writes the result and the solution.
void plain_begin(Problem& P, const cgl_node& nd, const NodeHost& nh, hipStream_t s) {
  PlainWork& W = P.plain;
  W.ensure(P);
  const int64_t p = P.p;
  // state, classes, initial iterate (ring slots 0 and 1 hold beta^0 = beta^1)
  NodeDev st0 = make_node_dev(nd, nh);
  CGL_HIP(hipMemcpyAsync(W.cls.ptr, nh.cls.data(), (size_t)p, hipMemcpyHostToDevice, s));
  CGL_HIP(hipMemsetAsync(W.bring.ptr, 0, 3 * P.ldx * 8, s));
  CGL_HIP(hipMemsetAsync(W.bbest.ptr, 0, P.ldx * 8, s));
  double L0_g = 0.0;
  if (nd.warm_start) {
    W.warm.assign(nd.warm_start, nd.warm_start + p);
    for (int64_t j = 0; j < p; ++j)
      if (nh.cls[(size_t)j] == CLS_ZERO) W.warm[(size_t)j] = 0.0;
    for (int slot = 0; slot < 2; ++slot)
      CGL_HIP(hipMemcpyAsync(W.bring.as<double>() + slot * P.ldx, W.warm.data(), p * 8,
                             hipMemcpyHostToDevice, s));
    L0_g = HUGE_VAL;  // the objective of an arbitrary start is not used for the restart test
  }
  W.st0 = st0;
  CGL_HIP(hipMemcpyAsync(W.st.ptr, &W.st0, sizeof(NodeDev), hipMemcpyHostToDevice, s));
  launch_xb(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, W.bring.as<double>() + P.ldx, 0,
            W.uring.as<double>() + P.n, 0, nullptr, P.y.as<double>(), P.loss,
            W.lpart.as<double>(), s);
  CGL_HIP(hipMemcpyAsync(W.uring.as<double>(), W.uring.as<double>() + P.n, P.n * 8,
                         hipMemcpyDeviceToDevice, s));
  launch_init_state(W.lpart.as<double>(), W.geom.nxb, L0_g, W.st.as<NodeDev>(), s);
  if (use_graphs() && !W.graph_exec) {
    hipGraph_t graph;
    CGL_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < PlainWork::kChunk; ++i) plain_iteration(P, W, s);
    CGL_HIP(hipStreamEndCapture(s, &graph));
    CGL_HIP(hipGraphInstantiate(&W.graph_exec, graph, nullptr, nullptr, 0));
    CGL_HIP(hipGraphDestroy(graph));
  }
  W.iter_before = 1;
}

void plain_launch(Problem& P, hipStream_t s) {
  PlainWork& W = P.plain;
  cgl_ctx* ctx = P.ctx;
  if (ctx->profiling) {
    for (int i = 0; i < PlainWork::kChunk; ++i) {
      hipEvent_t ev[4] = {ctx->event(4 * i), ctx->event(4 * i + 1), ctx->event(4 * i + 2),
                          ctx->event(4 * i + 3)};
      plain_iteration(P, W, s, ev);
    }
  } else if (W.graph_exec) {
    CGL_HIP(hipGraphLaunch(W.graph_exec, s));
  } else {
    for (int i = 0; i < PlainWork::kChunk; ++i) plain_iteration(P, W, s);
  }
  CGL_HIP(hipMemcpyAsync(W.st_host, W.st.ptr, sizeof(NodeDev), hipMemcpyDeviceToHost, s));
  CGL_HIP(hipEventRecord(W.chunk_ev, s));
}

bool plain_after_chunk(Problem& P) {
  PlainWork& W = P.plain;
  cgl_ctx* ctx = P.ctx;
  NodeDev* sh = W.st_host;
  if (ctx->profiling) {
    // only launches of iterations that ran (the rest returned at once) are counted
    const int ran = std::min(PlainWork::kChunk, sh->iter - W.iter_before);
    for (int i = 0; i < ran; ++i) {
      float a = 0.f, b = 0.f;
      CGL_HIP(hipEventElapsedTime(&a, ctx->event(4 * i), ctx->event(4 * i + 1)));
      CGL_HIP(hipEventElapsedTime(&b, ctx->event(4 * i + 2), ctx->event(4 * i + 3)));
      ctx->kt_ms[0] += a;
      ctx->kt_ms[1] += b;
      ctx->kt_n[0] += 1;
      ctx->kt_n[1] += 1;
    }
  }
  W.iter_before = sh->iter;
  return sh->done != 0;
}

void plain_end(Problem& P, cgl_result* res, double* beta_out, hipStream_t s) {
  PlainWork& W = P.plain;
  fill_result(*W.st_host, res);
  if (beta_out)
    CGL_HIP(hipMemcpyAsync(beta_out, W.bbest.ptr, P.p * 8, hipMemcpyDeviceToHost, s));
  CGL_HIP(hipStreamSynchronize(s));
}

void solve_plain(Problem& P, const cgl_node& nd, const NodeHost& nh, double* beta_out,
                 cgl_result* res) {
  if (P.plain.busy) invalid("the problem's FP64 path is in use by a server");
  hipStream_t s = P.ctx->stream;
  plain_begin(P, nd, nh, s);
  for (;;) {
    plain_launch(P, s);
    CGL_HIP(hipEventSynchronize(P.plain.chunk_ev));
    if (plain_after_chunk(P)) break;
  }
  plain_end(P, res, beta_out, s);
}

// ------------------------------------------------------------------ FP64 certificate at beta

void certify_host_beta(Problem& P, const NodeHost& nh, const double* beta, double* primal,
                       double* dual) {
  hipStream_t s = P.ctx->stream;
  const PlainGeom g = plain_geometry(P.xtype, P.n, P.ldx);
  DevBuf b, u, r, part, h, part2, cls, st, out;
  b.alloc(P.ldx * 8);
  u.alloc(P.n * 8);
  r.alloc(P.n * 8);
  part.alloc((size_t)g.nchunks * P.ldx * 8);
  h.alloc(P.ldx * 8);
  const int nb = (int)((P.n + 255) / 256);
  part2.alloc((size_t)nb * 16);
  cls.alloc(P.ldx);
  st.alloc(sizeof(NodeDev));
  out.alloc(16);
  CGL_HIP(hipMemsetAsync(b.ptr, 0, P.ldx * 8, s));
  CGL_HIP(hipMemcpyAsync(b.ptr, beta, P.p * 8, hipMemcpyHostToDevice, s));
  CGL_HIP(hipMemcpyAsync(cls.ptr, nh.cls.data(), P.p, hipMemcpyHostToDevice, s));
  NodeDev sd;
  std::memset(&sd, 0, sizeof(sd));
  sd.kp = nh.kp;
  sd.nfree = nh.nfree;
  CGL_HIP(hipMemcpyAsync(st.ptr, &sd, sizeof(sd), hipMemcpyHostToDevice, s));
  launch_xb(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, b.as<double>(), 0, u.as<double>(), 0, nullptr,
            nullptr, 0, nullptr, s);
  launch_resid(u.as<double>(), P.y.as<double>(), P.n, P.loss, r.as<double>(), part2.as<double>(),
               s);
  launch_xt(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, g, r.as<double>(), 0, nullptr, nullptr, 0, 1,
            part.as<double>(), nullptr, s);
  launch_grad_step(part.as<double>(), g.nchunks, P.ldx, nullptr, nullptr, 0, 0.0, h.as<double>(),
                   nullptr, s);
  launch_g_gstar(1, b.as<double>(), 0, h.as<double>(), 0, cls.as<uint8_t>(), 0,
                 st.as<NodeDev>(), P.p, P.M, 2.0 * P.lam2, out.as<double>(), s);
  std::vector<double> p2((size_t)nb * 2);
  double gg[2];
  CGL_HIP(hipMemcpyAsync(p2.data(), part2.ptr, (size_t)nb * 16, hipMemcpyDeviceToHost, s));
  CGL_HIP(hipMemcpyAsync(gg, out.ptr, 16, hipMemcpyDeviceToHost, s));
  CGL_HIP(hipStreamSynchronize(s));
  double f = 0.0, fs = 0.0;
  for (int i = 0; i < nb; ++i) { f += p2[(size_t)2 * i]; fs += p2[(size_t)2 * i + 1]; }
  *primal = std::isinf(gg[0]) ? HUGE_VAL : f + 2.0 * P.lam2 * gg[0];
  *dual = -fs - 2.0 * P.lam2 * gg[1];
}

}  // namespace cgl

using namespace cgl;

// ====================================================================== C ABI

extern "C" {

int cgl_version(void) { return CGL_ABI_VERSION; }

const char* cgl_status_str(int status) {
  switch (status) {
    case CGL_OK: return "ok";
    case CGL_E_INVAL: return "invalid argument";
    case CGL_E_NOMEM: return "out of memory";
    case CGL_E_DEVICE: return "device error";
    case CGL_E_BUSY: return "busy";
    case CGL_E_NOTFOUND: return "not found";
    case CGL_E_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

const char* cgl_last_error(void) { return g_last_error.c_str(); }

void cgl_node_init(cgl_node* node) {
  if (!node) return;
  std::memset(node, 0, sizeof(*node));
  node->tol = 1e-6;
  node->max_iter = 100000;
  node->check_every = 1;
  node->precision = CGL_PREC_F64;
  node->incumbent = HUGE_VAL;
}

int cgl_ctx_create(int device, void* hip_stream, cgl_ctx** out) {
  CGL_API_BEGIN
  if (!out) invalid("out is NULL");
  *out = nullptr;
  int ndev = 0;
  CGL_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) invalid("device ordinal out of range");
  CGL_HIP(hipSetDevice(device));
  noalloc_setup(device);  // this device's address of the allocation-free prox's scratch
  std::unique_ptr<cgl_ctx> c(new cgl_ctx());
  c->device = device;
  {
    hipDeviceProp_t prop;
    CGL_HIP(hipGetDeviceProperties(&prop, device));
    c->arch = prop.gcnArchName;
    const size_t colon = c->arch.find(':');
    if (colon != std::string::npos) c->arch.resize(colon);
    c->load_tuning();
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
    c->own_stream = false;
  } else {
    CGL_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  *out = c.release();
  return CGL_OK;
  CGL_API_END
}

int cgl_ctx_destroy(cgl_ctx* ctx) {
  CGL_API_BEGIN
  if (!ctx) return CGL_OK;
  (void)hipSetDevice(ctx->device);
  delete ctx;
  return CGL_OK;
  CGL_API_END
}

int cgl_ctx_set_profiling(cgl_ctx* ctx, int32_t on) {
  CGL_API_BEGIN
  if (!ctx) invalid("ctx is NULL");
  if (on < 0 || on > 3) invalid("profiling level must be 0, 1, 2 or 3");
  ctx->profiling = on == 1 || on == 2;
  ctx->profile_x = on == 2;
  ctx->phase_timing = on != 0;
  return CGL_OK;
  CGL_API_END
}

int cgl_ctx_kernel_stats(cgl_ctx* ctx, int32_t which, int32_t reset, double* total_ms,
                         int64_t* launches) {
  CGL_API_BEGIN
  if (!ctx) invalid("ctx is NULL");
  if (which < 0 || which >= 16) invalid("which out of range");
  if (which == 14) {  // the tilings in use (not counters: reset does not apply)
    if (total_ms) *total_ms = (double)ctx->tiling[0];
    if (launches) *launches = ctx->tiling[1];
    return CGL_OK;
  }
  if (total_ms) *total_ms = ctx->kt_ms[which];
  if (launches) *launches = ctx->kt_n[which];
  if (reset) {
    ctx->kt_ms[which] = 0.0;
    ctx->kt_n[which] = 0;
  }
  return CGL_OK;
  CGL_API_END
}

int cgl_node_validate(const cgl_node* node, int64_t p, int32_t k, int32_t* infeasible) {
  CGL_API_BEGIN
  if (!node) invalid("node is NULL");
  if (p < 1 || k < 1) invalid("p and k must be >= 1");
  const NodeHost h = make_node_host(*node, p, k);
  if (infeasible) *infeasible = h.infeasible ? 1 : 0;
  return CGL_OK;
  CGL_API_END
}

int cgl_problem_create(cgl_ctx* ctx, const void* X, int32_t x_dtype, int32_t x_mem, int64_t n,
                       int64_t p, int64_t ldx, const double* y, int32_t loss, double lambda2,
                       double M, int32_t k, double L, cgl_problem** out) {
  CGL_API_BEGIN
  // the arguments' values are checked before the context, so that these checks run (and can be
  // tested) without a device
  if (!out) invalid("out is NULL");
  *out = nullptr;
  if (!X || !y) invalid("X or y is NULL");
  if (n < 1 || p < 1) invalid("n and p must be >= 1");
  if (p > 32768) invalid("p > 32768 is not supported by this build");
  if (ldx < p) invalid("ldx < p");
  if (x_dtype != CGL_F64 && x_dtype != CGL_F32 && x_dtype != CGL_BF16) invalid("bad x_dtype");
  if (x_mem != CGL_MEM_HOST && x_mem != CGL_MEM_DEVICE) invalid("bad x_mem");
  if (loss < CGL_LOSS_LS || loss > CGL_LOSS_GAMMA) invalid("bad loss");
  if ((loss == CGL_LOSS_POISSON || loss == CGL_LOSS_GAMMA) && !(L > 0.0))
    invalid("the Poisson and Gamma losses have no global Lipschitz constant: give L > 0");
  if (!(lambda2 > 0.0) || !std::isfinite(lambda2)) invalid("lambda2 must be > 0");
  if (!(M > 0.0) || !std::isfinite(M)) invalid("M must be > 0");
  if (k < 1) invalid("k must be >= 1");
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(y[i])) invalid("non-finite y");
    if ((loss == CGL_LOSS_LOGISTIC || loss == CGL_LOSS_SQHINGE) && y[i] != 1.0 && y[i] != -1.0)
      invalid("classification labels must be -1 or +1");
    if (loss == CGL_LOSS_POISSON && y[i] < 0.0) invalid("Poisson responses must be >= 0");
    if (loss == CGL_LOSS_GAMMA && !(y[i] > 0.0)) invalid("Gamma responses must be > 0");
  }
  if (x_mem == CGL_MEM_HOST) {
    const int64_t nbad = count_nonfinite_host(X, x_dtype, n, p, ldx);
    if (nbad > 0) invalid("X has " + std::to_string(nbad) + " non-finite entries");
  }
  if (!ctx) invalid("ctx is NULL");
  CGL_HIP(hipSetDevice(ctx->device));
  std::unique_ptr<Problem> P(new Problem());
  P->ctx = ctx;
  P->n = n;
  P->p = p;
  P->ldx = pad_cols(p);
  P->xtype = x_dtype == CGL_F64 ? XT_F64 : (x_dtype == CGL_F32 ? XT_F32 : XT_BF16);
  P->loss = loss;  // enum cgl_loss and LossKind share their values
  P->lam2 = lambda2;
  P->M = M;
  P->k = k;
  upload_X(*P, X, x_mem, ldx);
  if (x_mem == CGL_MEM_DEVICE) {
    // non-finite entries of a device X, counted on the device copy
    DevBuf bad;
    bad.alloc(sizeof(int));
    int nbad = 0;
    CGL_HIP(hipMemsetAsync(bad.ptr, 0, sizeof(int), ctx->stream));
    launch_count_nonfinite(P->xtype, P->X.ptr, n * P->ldx, bad.as<int>(), ctx->stream);
    CGL_HIP(hipMemcpyAsync(&nbad, bad.ptr, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    CGL_HIP(hipStreamSynchronize(ctx->stream));
    if (nbad > 0) invalid("X has " + std::to_string(nbad) + " non-finite entries");
  }
  P->y.alloc((size_t)n * 8);
  CGL_HIP(hipMemcpy(P->y.ptr, y, (size_t)n * 8, hipMemcpyHostToDevice));
  if (L > 0.0) {
    P->L = L;
  } else {
    const double lam = power_lambda_max(*P);
    const double factor = loss_lipschitz_factor(P->loss);
    P->lam_max = lam;
    P->L = factor * lam * 1.002;
  }
  P->rho = P->L / (2.0 * P->lam2);
  *out = reinterpret_cast<cgl_problem*>(P.release());
  return CGL_OK;
  CGL_API_END
}

int cgl_problem_share_design(cgl_problem* owner, cgl_problem* sharer) {
  CGL_API_BEGIN
  if (!owner || !sharer) invalid("NULL argument");
  Problem& O = *reinterpret_cast<Problem*>(owner);
  Problem& Q = *reinterpret_cast<Problem*>(sharer);
  if (&O == &Q) invalid("a problem cannot share its own design");
  if (O.ctx != Q.ctx) invalid("the problems belong to different contexts");
  if (O.n != Q.n || O.p != Q.p || O.xtype != Q.xtype)
    invalid("the problems differ in n, p or the stored precision of X");
  if (O.design_owner || Q.design_owner || !Q.sharers.empty())
    invalid("a problem already shares a design (one owner, sharers of that owner only)");
  if (O.sharers.size() + 1 >= (size_t)kMaxMembers)
    invalid("too many problems on one design (at most " + std::to_string(kMaxMembers) + ")");
  if (O.mixed || Q.mixed)
    invalid("a batched engine of either problem exists already: share before the first "
            "mixed-precision solve");
  CGL_HIP(hipSetDevice(O.ctx->device));
  DevBuf diff;
  diff.alloc(sizeof(int));
  int ndiff = 0;
  const int64_t bytes = O.n * O.ldx * (O.xtype == XT_F64 ? 8 : (O.xtype == XT_F32 ? 4 : 2));
  CGL_HIP(hipMemsetAsync(diff.ptr, 0, sizeof(int), O.ctx->stream));
  launch_count_diff(O.X.ptr, Q.X.ptr, bytes / 4, diff.as<int>(), O.ctx->stream);
  CGL_HIP(hipMemcpyAsync(&ndiff, diff.ptr, sizeof(int), hipMemcpyDeviceToHost, O.ctx->stream));
  CGL_HIP(hipStreamSynchronize(O.ctx->stream));
  if (ndiff != 0) invalid("the problems' designs differ");
  O.sharers.push_back(&Q);
  Q.design_owner = &O;
  return CGL_OK;
  CGL_API_END
}

int cgl_problem_destroy(cgl_problem* prob) {
  CGL_API_BEGIN
  if (!prob) return CGL_OK;
  Problem* P = reinterpret_cast<Problem*>(prob);
  (void)hipSetDevice(P->ctx->device);
  if (Problem* O = P->design_owner) {
    // the owner's engine keeps its copies of P's labels; it stops naming P
    O->sharers.erase(std::remove(O->sharers.begin(), O->sharers.end(), P), O->sharers.end());
    if (O->mixed) O->mixed->forget_member(P);
  }
  for (Problem* Q : P->sharers) Q->design_owner = nullptr;  // standalone from now on
  delete P;
  return CGL_OK;
  CGL_API_END
}

int cgl_problem_lipschitz(const cgl_problem* prob, double* L) {
  CGL_API_BEGIN
  if (!prob || !L) invalid("NULL argument");
  *L = reinterpret_cast<const Problem*>(prob)->L;
  return CGL_OK;
  CGL_API_END
}

int cgl_solve_node(cgl_problem* prob, const cgl_node* node, double* beta_out, cgl_result* res) {
  CGL_API_BEGIN
  if (!prob || !node || !res) invalid("NULL argument");
  Problem& P = *reinterpret_cast<Problem*>(prob);
  CGL_HIP(hipSetDevice(P.ctx->device));
  const NodeHost nh = make_node_host(*node, P.p, P.k);
  if (nh.infeasible) {
    infeasible_result(res, beta_out, P.p);
    return CGL_OK;
  }
  if (node->precision == CGL_PREC_MIXED) {
    solve_mixed(P, node, 1, beta_out, res);
  } else {
    solve_plain(P, *node, nh, beta_out, res);
  }
  return CGL_OK;
  CGL_API_END
}

int cgl_problem_set_eigen(cgl_problem* prob, double shift) {
  CGL_API_BEGIN
  if (!prob) invalid("prob is NULL");
  Problem& P = *reinterpret_cast<Problem*>(prob);
  if (P.loss != LOSS_LS) invalid("the eigen-perspective relaxation is for least squares");
  if (!(shift >= 0.0) || !std::isfinite(shift)) invalid("shift must be >= 0");
  const Problem& E = P.engine_problem();
  if ((E.mixed && (E.mixed->in_flight || E.mixed->free_slots() != E.mixed->S)) || P.plain.busy)
    invalid("a server runs nodes of the problem or of one sharing its design");
  CGL_HIP(hipSetDevice(P.ctx->device));
  if (P.lam_max <= 0.0) P.lam_max = power_lambda_max(P);
  if (shift >= P.lam_max) invalid("shift must be below lambda_max(X^T X)");
  if (!eigen_shift_proved(P, shift))
    invalid(P.n < P.p ? "X^T X is singular (n < p): only shift 0 is valid"
                      : "shift not certified: an FP64 Cholesky factorisation of X^T X - (shift + "
                        "rounding margin) I fails, so shift <= lambda_min(X^T X) is not proved");
  // L = 2 lambda_max(Q), Q = X^T X - s I, with the same safety factor on lambda_max; a graph
  // captured with the previous parameters is dropped
  if (P.plain.graph_exec) {
    CGL_HIP(hipGraphExecDestroy(P.plain.graph_exec));
    P.plain.graph_exec = nullptr;
  }
  P.shift = shift;
  P.L = 2.0 * (1.002 * P.lam_max - shift);
  P.rho = P.L / (2.0 * (P.lam2 + shift));
  return CGL_OK;
  CGL_API_END
}

int cgl_problem_eigen_shift(cgl_problem* prob, double* shift) {
  CGL_API_BEGIN
  if (!prob || !shift) invalid("NULL argument");
  Problem& P = *reinterpret_cast<Problem*>(prob);
  if (P.loss != LOSS_LS) invalid("the eigen-perspective relaxation is for least squares");
  CGL_HIP(hipSetDevice(P.ctx->device));
  if (P.lam_max <= 0.0) P.lam_max = power_lambda_max(P);
  *shift = eigen_shift_certified(P, 1e-7);
  return CGL_OK;
  CGL_API_END
}

static int solve_batch_impl(cgl_problem* prob, const cgl_node* nodes, int32_t count,
                            double* beta_out, cgl_result* res, double* dual_out) {
  CGL_API_BEGIN
  if (!prob || (count > 0 && (!nodes || !res))) invalid("NULL argument");
  if (count < 0) invalid("count < 0");
  Problem& P = *reinterpret_cast<Problem*>(prob);
  CGL_HIP(hipSetDevice(P.ctx->device));
  // validate everything before any work
  std::vector<NodeHost> hosts;
  hosts.reserve((size_t)count);
  for (int32_t i = 0; i < count; ++i) hosts.push_back(make_node_host(nodes[i], P.p, P.k));
  std::vector<cgl_node> mixed;
  std::vector<int32_t> mixed_idx;
  for (int32_t i = 0; i < count; ++i) {
    double* bo = beta_out ? beta_out + (int64_t)i * P.p : nullptr;
    if (dual_out && (hosts[(size_t)i].infeasible || nodes[i].precision != CGL_PREC_MIXED))
      std::fill(dual_out + (int64_t)i * P.p, dual_out + (int64_t)(i + 1) * P.p, std::nan(""));
    if (hosts[(size_t)i].infeasible) {
      infeasible_result(&res[i], bo, P.p);
    } else if (nodes[i].precision == CGL_PREC_MIXED) {
      mixed.push_back(nodes[i]);
      mixed_idx.push_back(i);
    } else {
      solve_plain(P, nodes[i], hosts[(size_t)i], bo, &res[i]);
    }
  }
  // the batched engine writes each node's result and solution straight into the caller's row
  if (!mixed.empty())
    solve_mixed(P, mixed.data(), (int32_t)mixed.size(), beta_out, res, mixed_idx.data(),
                dual_out);
  return CGL_OK;
  CGL_API_END
}

int cgl_solve_batch(cgl_problem* prob, const cgl_node* nodes, int32_t count, double* beta_out,
                    cgl_result* res) {
  return solve_batch_impl(prob, nodes, count, beta_out, res, nullptr);
}

int cgl_solve_batch_dual(cgl_problem* prob, const cgl_node* nodes, int32_t count,
                         double* beta_out, cgl_result* res, double* dual_beta_out) {
  if (!dual_beta_out && count > 0) {
    set_error("dual_beta_out is NULL");
    return CGL_E_INVAL;
  }
  return solve_batch_impl(prob, nodes, count, beta_out, res, dual_beta_out);
}

int cgl_certify(cgl_problem* prob, const cgl_node* node, const double* beta, double* primal,
                double* dual) {
  CGL_API_BEGIN
  if (!prob || !node || !beta || !primal || !dual) invalid("NULL argument");
  Problem& P = *reinterpret_cast<Problem*>(prob);
  if (P.shift != 0.0) invalid("cgl_certify evaluates the perspective relaxation (shift 0)");
  CGL_HIP(hipSetDevice(P.ctx->device));
  const NodeHost nh = make_node_host(*node, P.p, P.k);
  if (nh.infeasible) {
    *primal = HUGE_VAL;
    *dual = HUGE_VAL;
    return CGL_OK;
  }
  for (int64_t j = 0; j < P.p; ++j)
    if (!std::isfinite(beta[j])) invalid("non-finite beta");
  certify_host_beta(P, nh, beta, primal, dual);
  return CGL_OK;
  CGL_API_END
}

int cgl_problem_matvec(cgl_problem* prob, int32_t trans, const double* v, double* out) {
  CGL_API_BEGIN
  if (!prob || !v || !out) invalid("NULL argument");
  if (trans != 0 && trans != 1) invalid("trans must be 0 or 1");
  Problem& P = *reinterpret_cast<Problem*>(prob);
  CGL_HIP(hipSetDevice(P.ctx->device));
  hipStream_t s = P.ctx->stream;
  DevBuf in, o;
  if (trans == 0) {
    in.alloc(P.ldx * 8);
    o.alloc(P.n * 8);
    CGL_HIP(hipMemsetAsync(in.ptr, 0, P.ldx * 8, s));
    CGL_HIP(hipMemcpyAsync(in.ptr, v, P.p * 8, hipMemcpyHostToDevice, s));
    launch_xb(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, in.as<double>(), 0, o.as<double>(), 0,
              nullptr, nullptr, 0, nullptr, s);
    CGL_HIP(hipMemcpyAsync(out, o.ptr, P.n * 8, hipMemcpyDeviceToHost, s));
  } else {
    const PlainGeom g = plain_geometry(P.xtype, P.n, P.ldx);
    DevBuf part;
    in.alloc(P.n * 8);
    o.alloc(P.ldx * 8);
    part.alloc((size_t)g.nchunks * P.ldx * 8);
    CGL_HIP(hipMemcpyAsync(in.ptr, v, P.n * 8, hipMemcpyHostToDevice, s));
    launch_xt(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, g, in.as<double>(), 0, nullptr, nullptr, 0, 1,
              part.as<double>(), nullptr, s);
    launch_grad_step(part.as<double>(), g.nchunks, P.ldx, nullptr, nullptr, 0, 0.0,
                     o.as<double>(), nullptr, s);
    CGL_HIP(hipMemcpyAsync(out, o.ptr, P.p * 8, hipMemcpyDeviceToHost, s));
  }
  CGL_HIP(hipStreamSynchronize(s));
  return CGL_OK;
  CGL_API_END
}

int cgl_prox_node_batch(cgl_ctx* ctx, double rho, double M, int32_t k, const cgl_node* nodes,
                        const double* W, int32_t count, int64_t p, double* beta_out,
                        double* gval_out) {
  CGL_API_BEGIN
  if (!ctx || !W || !beta_out) invalid("NULL argument");
  if (count < 0 || p < 1) invalid("count < 0 or p < 1");
  if (p > kProxMaxP) invalid("p > 1048576 is not supported by this build");
  if (!(rho > 0.0) || !(M > 0.0) || k < 0) invalid("need rho > 0, M > 0, k >= 0");
  if (count == 0) return CGL_OK;
  CGL_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  std::vector<uint8_t> cls((size_t)count * p, CLS_FREE);
  std::vector<NodeDev> st((size_t)count);
  std::vector<int> infeasible((size_t)count, 0);
  for (int32_t i = 0; i < count; ++i) {
    cgl_node nd;
    cgl_node_init(&nd);
    if (nodes) nd = nodes[i];
    NodeHost h = make_node_host(nd, p, k);
    std::copy(h.cls.begin(), h.cls.end(), cls.begin() + (int64_t)i * p);
    NodeDev sd = make_node_dev(nd, h);
    sd.kp = std::max(h.kp, 0);
    sd.check_every = 1 << 30;
    sd.max_iter = 1 << 30;
    st[(size_t)i] = sd;
    infeasible[(size_t)i] = h.infeasible;
  }
  DevBuf dW, dB, dC, dS;
  dW.alloc((size_t)count * p * 8);
  dB.alloc((size_t)count * p * 8);
  dC.alloc((size_t)count * p);
  dS.alloc((size_t)count * sizeof(NodeDev));
  CGL_HIP(hipMemcpyAsync(dW.ptr, W, (size_t)count * p * 8, hipMemcpyHostToDevice, s));
  CGL_HIP(hipMemcpyAsync(dC.ptr, cls.data(), (size_t)count * p, hipMemcpyHostToDevice, s));
  CGL_HIP(hipMemcpyAsync(dS.ptr, st.data(), (size_t)count * sizeof(NodeDev),
                         hipMemcpyHostToDevice, s));
  if (ctx->profiling) CGL_HIP(hipEventRecord(ctx->event(0), s));
  // up to 16 values per thread in the workgroup's LDS slices; beyond that the register-held
  // variants spill, and the kernel that streams each vector from memory is faster (256 against
  // about 140 us for one vector at p = 25600)
  if (p <= kProxHeldP)
    launch_prox(count, dW.as<double>(), p, nullptr, 0, dC.as<uint8_t>(), p, p, rho, M, 1.0,
                dS.as<NodeDev>(), dB.as<double>(), 0, p, s);
  else
    launch_prox_paged(count, dW.as<double>(), p, dC.as<uint8_t>(), p, p, rho, M,
                      dS.as<NodeDev>(), dB.as<double>(), p, s);
  if (ctx->profiling) CGL_HIP(hipEventRecord(ctx->event(1), s));
  CGL_HIP(hipMemcpyAsync(beta_out, dB.ptr, (size_t)count * p * 8, hipMemcpyDeviceToHost, s));
  CGL_HIP(hipMemcpyAsync(st.data(), dS.ptr, (size_t)count * sizeof(NodeDev),
                         hipMemcpyDeviceToHost, s));
  CGL_HIP(hipStreamSynchronize(s));
  if (ctx->profiling) {
    float ms = 0.f;
    CGL_HIP(hipEventElapsedTime(&ms, ctx->event(0), ctx->event(1)));
    ctx->kt_ms[8] += ms;
    ctx->kt_n[8] += 1;
  }
  if (gval_out)
    for (int32_t i = 0; i < count; ++i)
      gval_out[i] = infeasible[(size_t)i] ? HUGE_VAL : st[(size_t)i].g_new;
  return CGL_OK;
  CGL_API_END
}

}  // extern "C"

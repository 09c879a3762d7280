// Batched mixed-precision engine: node slots sharing one X, BF16 MFMA correction products around
// FP64 base points, batched FP64 re-centring / certification rounds, and continuous refill of
// finished slots from a queue (used by cgl_solve_batch, cgl_solve_node with CGL_PREC_MIXED and
// the server).
#include "batch.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "common.h"
#include "engine.h"
#include "gemm_bf16.h"
#include "kernels.h"
#include "losses.h"
#include "mixed.h"
#include "prox.h"

namespace cgl {

Problem::~Problem() { delete mixed; }

MixedWork::~MixedWork() {
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (st_host) (void)hipHostFree(st_host);
  if (beta_host) (void)hipHostFree(beta_host);
  if (count_host) (void)hipHostFree(count_host);
  if (order_host) (void)hipHostFree(order_host);
  if (cls_host) (void)hipHostFree(cls_host);
  if (list_host) (void)hipHostFree(list_host);
  if (ret_gathered) (void)hipEventDestroy(ret_gathered);
  if (ret_copied) (void)hipEventDestroy(ret_copied);
  if (copy_stream) (void)hipStreamDestroy(copy_stream);
  if (chunk_done) (void)hipEventDestroy(chunk_done);
}

static int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

void MixedWork::ensure(Problem& P) {
  if (ready) return;
  if (!stream) stream = P.ctx->stream;
  hipStream_t s = stream;
  std::fill(want_since, want_since + kSlots, (int64_t)-1);
  // batching of the certification rounds (tuning knobs; the defaults suit the 256-slot engine)
  for (auto [name, dst] : {std::pair<const char*, int*>{"CGL_CERT_BATCH", &cert_batch},
                           std::pair<const char*, int*>{"CGL_CERT_WAIT", &cert_wait},
                           std::pair<const char*, int*>{"CGL_REORDER_EVERY", &reorder_every},
                           std::pair<const char*, int*>{"CGL_REORDER_SHRINK", &reorder_shrink}}) {
    const char* e = std::getenv(name);
    if (e && std::atoi(e) > 0) *dst = std::atoi(e);
  }
  {
    const char* e = std::getenv("CGL_CHUNK");
    if (e && std::atoi(e) > 0) serve_chunk = solve_chunk = std::atoi(e);
  }
  // the timing events of a chunk (4 per cycle) stay below those of the FP64 rounds
  serve_chunk = std::min(serve_chunk, 16);
  solve_chunk = std::min(solve_chunk, 16);
  chunk = serve_chunk;
  // the problems the engine serves: its own and those declared to share its design
  members.assign(1, &P);
  for (Problem* Q : P.sharers) members.push_back(Q);
  bool any_ls = false, any_other = false;
  for (Problem* Q : members) (Q->loss == LOSS_LS ? any_ls : any_other) = true;
  S = kSlots;
  S_pad = (int)round_up(S, 256);
  n_pad = round_up(P.n, GT_M);  // rows of X~: a multiple of the GEMM tile and of its k-chunk grain
  ldp = P.ldx;
  // BF16 design and its transpose
  Xb.alloc((size_t)n_pad * ldp * 2);
  Xbt.alloc((size_t)ldp * n_pad * 2);
  launch_make_bf16(P.xtype, P.X.ptr, P.ldx, P.n, P.p, n_pad, ldp, Xb.as<uint16_t>(),
                   Xbt.as<uint16_t>(), s);
  mbufs.clear();
  for (Problem* Q : members) {
    mbufs.emplace_back(new MemberBufs());
    DevBuf& yp = mbufs.back()->y;
    yp.alloc((size_t)n_pad * 8);
    CGL_HIP(hipMemsetAsync(yp.ptr, 0, (size_t)n_pad * 8, s));
    CGL_HIP(hipMemcpyAsync(yp.ptr, Q->y.ptr, (size_t)P.n * 8, hipMemcpyDeviceToDevice, s));
  }
  // slots
  const size_t Sp = (size_t)S * ldp, Sn = (size_t)S * n_pad;
  st.alloc(st_bytes());
  cls.alloc(Sp);
  bring.alloc(3 * Sp * 8);
  beta0.alloc(Sp * 8);
  H0.alloc(Sp * 8);
  base0.alloc(any_other ? Sn * 8 : 8);
  base1.alloc(any_other ? Sn * 8 : 8);
  e0f.alloc(any_ls ? Sn * 4 : 8);
  bres.alloc(Sp * 8);
  bdual.alloc(Sp * 8);
  dop.alloc((size_t)S_pad * ldp * 2);
  gop.alloc((size_t)S_pad * n_pad * 2);
  gop_r.alloc((size_t)S_pad * n_pad * 2);
  gsel.alloc((size_t)S_pad * sizeof(int));
  dU.alloc(2 * (size_t)S_pad * n_pad * 4);
  // split-K of the two products: the candidates keep >= 16 k-steps of 32 per chunk and at most
  // four rounds of 256 workgroups (one workgroup of the product fits on a compute unit); the
  // partial buffers are sized for the largest candidate and the choice is made by timing
  // (tune_splits) once the buffers exist
  split_cands_x = tiling_candidates(n_pad, ldp);
  split_cands_xt = tiling_candidates(ldp, n_pad);
  set_split_x(split_cands_x.front());
  set_split_xt(split_cands_xt.front());
  {
    int kx = 1, kt = 1;
    for (int c : split_cands_x) kx = std::max(kx, code_ks(c));
    for (int c : split_cands_xt) kt = std::max(kt, code_ks(c));
    dUp.alloc((size_t)kx * S_pad * n_pad * 4);
    dH.alloc((size_t)kt * S_pad * ldp * 4);
  }
  rchunk = kLossChunk;
  nrt = (int)((n_pad + rchunk - 1) / rchunk);
  lpart.alloc((size_t)S * nrt * 8);
  npart.alloc((size_t)S * nrt * 8);
  fpart.alloc((size_t)S * 2 * nrt * 8);
  cycle.alloc(sizeof(int));
  CGL_HIP(hipMemsetAsync(cycle.ptr, 0xff, sizeof(int), s));  // -1: the first cycle is 0
  prevsel.alloc((size_t)2 * S * 65 * sizeof(int));
  CGL_HIP(hipMemsetAsync(prevsel.ptr, 0, prevsel.bytes, s));
  CGL_HIP(hipMemsetAsync(dop.ptr, 0, (size_t)S_pad * ldp * 2, s));
  CGL_HIP(hipMemsetAsync(gop.ptr, 0, (size_t)S_pad * n_pad * 2, s));
  CGL_HIP(hipMemsetAsync(gop_r.ptr, 0, (size_t)S_pad * n_pad * 2, s));
  CGL_HIP(hipMemsetAsync(gsel.ptr, 0, gsel.bytes, s));
  CGL_HIP(hipMemsetAsync(dU.ptr, 0, 2 * (size_t)S_pad * n_pad * 4, s));
  CGL_HIP(hipMemsetAsync(dH.ptr, 0, dH.bytes, s));
  // certification buffers
  B64.alloc(Sp * 8);
  U64.alloc(Sn * 8);
  R64.alloc(Sn * 8);
  H64.alloc(Sp * 8);
  CGL_HIP(hipMemsetAsync(H64.ptr, 0, Sp * 8, s));
  CGL_HIP(hipMemsetAsync(U64.ptr, 0, Sn * 8, s));
  // union of the certified iterates' supports: flags (zero between rounds), the list, its size
  // and the iterates compacted to it
  sflag.alloc((size_t)ldp);
  CGL_HIP(hipMemsetAsync(sflag.ptr, 0, (size_t)ldp, s));
  sidx.alloc((size_t)ldp * sizeof(int));
  scount.alloc(sizeof(int));
  Bu.alloc(Sp * 8);
  // split-K partials of the FP64 products (split x nodes <= 2 S)
  part64_cap = 2 * (size_t)S * (size_t)std::max<int64_t>(n_pad, ldp) * 8;
  part64.alloc(part64_cap);
  // X^T in the stored precision for the FP64 X^T products (the BF16 transpose is exact for BF16)
  if (P.xtype != XT_BF16) {
    Xt.alloc((size_t)P.p * n_pad * (P.xtype == XT_F64 ? 8 : 4));
    launch_transpose(P.xtype, P.X.ptr, P.ldx, P.n, P.p, n_pad, Xt.ptr, s);
  }
  cchunk = 2048;
  ncchunk = (int)((n_pad + cchunk - 1) / cchunk);
  cpart.alloc((size_t)S * ncchunk * 16);
  list.alloc((size_t)S * sizeof(int));
  // cold-start base of each problem: u_0 = 0, r_0 = grad f(0) = a + b y (per loss), H_0 = X^T r_0
  // in FP64
  for (size_t m = 0; m < members.size(); ++m) {
    const Problem& Q = *members[m];
    MemberBufs& B = *mbufs[m];
    const PlainGeom g = plain_geometry(P.xtype, P.n, P.ldx);
    std::vector<double> yv((size_t)P.n), r0((size_t)P.n);
    CGL_HIP(hipMemcpy(yv.data(), Q.y.ptr, (size_t)P.n * 8, hipMemcpyDeviceToHost));
    const double ga = loss_grad0_a(Q.loss), gb = loss_grad0_b(Q.loss);
    for (int64_t i = 0; i < P.n; ++i) r0[(size_t)i] = ga + gb * yv[(size_t)i];
    DevBuf part, dr0;
    part.alloc((size_t)g.nchunks * P.ldx * 8);
    dr0.alloc((size_t)P.n * 8);
    CGL_HIP(hipMemcpy(dr0.ptr, r0.data(), (size_t)P.n * 8, hipMemcpyHostToDevice));
    B.H0c.alloc((size_t)ldp * 8);
    CGL_HIP(hipMemsetAsync(B.H0c.ptr, 0, (size_t)ldp * 8, s));
    launch_xt(P.xtype, P.X.ptr, P.ldx, P.n, P.ldx, g, dr0.as<double>(), 0, nullptr, nullptr, 0,
              1, part.as<double>(), nullptr, s);
    launch_grad_step(part.as<double>(), g.nchunks, P.ldx, nullptr, nullptr, 0, 0.0,
                     B.H0c.as<double>(), nullptr, s);
    CGL_HIP(hipStreamSynchronize(s));
    std::vector<double> b0((size_t)n_pad, 0.0), b1((size_t)n_pad, 0.0);
    for (int64_t i = 0; i < P.n; ++i) {
      if (Q.loss == LOSS_LS) b0[(size_t)i] = -yv[(size_t)i];  // e_0 = 0 - y
      else b1[(size_t)i] = r0[(size_t)i];                      // r_0, with u_0 = 0
    }
    B.b0c.alloc((size_t)n_pad * 8);
    B.b1c.alloc((size_t)n_pad * 8);
    CGL_HIP(hipMemcpy(B.b0c.ptr, b0.data(), (size_t)n_pad * 8, hipMemcpyHostToDevice));
    CGL_HIP(hipMemcpy(B.b1c.ptr, b1.data(), (size_t)n_pad * 8, hipMemcpyHostToDevice));
  }
  // Least squares with n >= p: G = X^T X in FP64 (2 n p^2 FLOP, once per engine), so that a
  // certification round gets X^T grad f(X beta) = 2 G beta - 2 X^T y from the rows of G on the
  // union of the iterates' supports instead of a product with all of X. CGL_NO_GRAM=1 turns it
  // off.
  {
    const char* ng = std::getenv("CGL_NO_GRAM");
    if (any_ls && P.n >= P.p && P.p <= kGramMaxP && !(ng && std::atoi(ng) > 0)) {
      ldg = round_up(P.p, 256);
      G.alloc((size_t)P.p * ldg * 8);
      CGL_HIP(hipMemsetAsync(G.ptr, 0, G.bytes, s));
      build_gram(P.xtype, P.xtype == XT_BF16 ? Xbt.ptr : Xt.ptr, n_pad, P.n, P.p,
                 G.as<double>(), ldg, part64.as<double>(), part64_cap, s);
    }
  }
  CGL_HIP(hipHostMalloc(&st_host, st_bytes(), hipHostMallocDefault));
  CGL_HIP(hipHostMalloc(&beta_host, (size_t)S * P.p * sizeof(double), hipHostMallocDefault));
  CGL_HIP(hipHostMalloc(&count_host, sizeof(int), hipHostMallocDefault));
  Bret.alloc((size_t)S * P.p * sizeof(double));
  CGL_HIP(hipStreamCreateWithFlags(&copy_stream, hipStreamNonBlocking));
  CGL_HIP(hipEventCreateWithFlags(&ret_gathered, hipEventDisableTiming));
  CGL_HIP(hipEventCreateWithFlags(&ret_copied, hipEventDisableTiming));
  CGL_HIP(hipEventCreateWithFlags(&chunk_done, hipEventDisableTiming));
  std::memset(st_host, 0, st_bytes());
  CGL_HIP(hipMemcpyAsync(st.ptr, st_host, st_bytes(), hipMemcpyHostToDevice, s));
  CGL_HIP(hipHostMalloc(&cls_host, Sp, hipHostMallocDefault));
  std::memset(cls_host, CLS_PAD, Sp);
  CGL_HIP(hipHostMalloc(&list_host, 3 * (size_t)S * sizeof(int), hipHostMallocDefault));
  slot_owner.assign((size_t)S, -1);
  // device view
  md.Xb = Xb.as<uint16_t>();
  md.Xbt = Xbt.as<uint16_t>();
  md.n = P.n;
  md.p = P.p;
  md.n_pad = n_pad;
  md.ldp = ldp;
  memtab.alloc(kMaxMembers * sizeof(MemberDev));
  for (size_t m = 0; m < members.size(); ++m) {
    MemberDev& d = mem_host[m];
    const Problem& Q = *members[m];
    d.y = mbufs[m]->y.as<double>();
    d.H0c = mbufs[m]->H0c.as<double>();
    d.b0c = mbufs[m]->b0c.as<double>();
    d.b1c = mbufs[m]->b1c.as<double>();
    d.loss = Q.loss;
    d.lam2 = Q.lam2;
    d.M = Q.M;
    d.L = Q.L;
    d.rho = Q.rho;
    d.shift = Q.shift;
  }
  CGL_HIP(hipMemcpyAsync(memtab.ptr, mem_host, sizeof(mem_host), hipMemcpyHostToDevice, s));
  md.mem = memtab.as<MemberDev>();
  md.cert_gap = kCertGap;
  md.stall_cycles = kStallCycles;
  {  // tuning knobs of the certification requests (defaults: the fastest of a sweep on the
     // 256-node least-squares workload)
    const char* g = std::getenv("CGL_CERT_GAP");
    if (g && std::atof(g) > 0.0) md.cert_gap = std::atof(g);
    const char* c = std::getenv("CGL_STALL_CYCLES");
    if (c && std::atoi(c) > 0) md.stall_cycles = std::atoi(c);
    md.restart_slack = kRestartSlack;
    const char* r = std::getenv("CGL_RESTART_SLACK");
    if (r && std::atof(r) >= 0.0) md.restart_slack = std::atof(r);
  }
  md.slots = S;
  md.S_pad = S_pad;
  md.st = st.as<NodeDev>();
  md.cls = cls.as<uint8_t>();
  md.bring = bring.as<double>();
  md.bring_stride = (int64_t)Sp;
  md.beta0 = beta0.as<double>();
  md.H0 = H0.as<double>();
  md.base0 = base0.as<double>();
  md.base1 = base1.as<double>();
  md.e0f = e0f.as<float>();
  md.bres = bres.as<double>();
  md.bdual = bdual.as<double>();
  md.dop = dop.as<uint16_t>();
  md.gop = gop.as<uint16_t>();
  md.gop_r = gop_r.as<uint16_t>();
  md.gsel = gsel.as<int>();
  md.dU = dU.as<float>();
  md.dU_ring = (int64_t)S_pad * n_pad;
  md.dUp = dUp.as<float>();
  md.dUp_split = (int64_t)S_pad * n_pad;
  md.ksx = ksx;
  md.x_kchunk = x_kchunk;
  md.dH = dH.as<float>();
  md.dH_split = (int64_t)S_pad * ldp;
  md.ksplit = ksplit;
  md.xt_kchunk = xt_kchunk;
  md.lpart = lpart.as<double>();
  md.npart = npart.as<double>();
  md.fpart = fpart.as<double>();
  md.nrt = nrt;
  md.loss_kinds = (any_ls ? 1 : 0) | (any_other ? 2 : 0);
  md.rchunk = rchunk;
  md.cycle = cycle.as<int>();
  md.prevhead = prevsel.as<int>();
  md.prevtop = prevsel.as<int>() + (size_t)S * 65;
  // X-pass operand order: identity until the first reorder; full extent until the node kernels
  // have measured it
  {
    std::vector<int> id((size_t)ldp);
    for (int64_t j = 0; j < ldp; ++j) id[(size_t)j] = (int)j;
    pinv.alloc((size_t)ldp * sizeof(int));
    pinv_new.alloc((size_t)ldp * sizeof(int));
    perm.alloc((size_t)ldp * sizeof(int));
    perm_new.alloc((size_t)ldp * sizeof(int));
    CGL_HIP(hipMemcpy(pinv.ptr, id.data(), (size_t)ldp * sizeof(int), hipMemcpyHostToDevice));
    CGL_HIP(hipMemcpy(perm.ptr, id.data(), (size_t)ldp * sizeof(int), hipMemcpyHostToDevice));
    // the extent counters start at the full width (the strays per slot at zero, as the state)
    int* tail = ctl_dev();
    int* th = (int*)((char*)st_host + (size_t)S * sizeof(NodeDev));
    th[kCtlExtent] = th[kCtlExtent + 1] = (int)ldp;
    CGL_HIP(hipMemcpyAsync(tail, th, 2 * sizeof(int), hipMemcpyHostToDevice, s));  // after the zeros
    dop_tmp.alloc(dop.bytes);
    CGL_HIP(hipHostMalloc(&order_host, sizeof(int), hipHostMallocDefault));
    // no support prefix (and so no strays) until the first reorder
    pfx.alloc(sizeof(int));
    const int nopfx = (int)ldp;
    CGL_HIP(hipMemcpy(pfx.ptr, &nopfx, sizeof(int), hipMemcpyHostToDevice));
    sj.alloc((size_t)S * kStrayCap * sizeof(int));
    sv.alloc((size_t)S * kStrayCap * sizeof(float));
    md.pfx = pfx.as<int>();
    md.sn = tail + kCtlStrays;
    md.sj = sj.as<int>();
    md.sv = sv.as<float>();
    const char* e = std::getenv("CGL_NO_REORDER");
    reorder = !(e && std::atoi(e) > 0);
    // test hook: a support prefix shorter than the union (multiple of 128) forces strays and
    // operand entries past the prefix
    const char* c = std::getenv("CGL_PREFIX_CAP");
    if (c && std::atoi(c) > 0) prefix_cap = round_up(std::atoi(c), 2 * GT_K);
    md.pinv = pinv.as<int>();
    md.perm = perm.as<int>();
    md.keff = tail + kCtlExtent;
  }
  CGL_HIP(hipStreamSynchronize(s));
  tune_splits(P);
  ready = true;
}

void MixedWork::set_relaxation(Problem& P) {
  (void)P;
  bool changed = false;
  for (size_t m = 0; m < members.size(); ++m) {
    if (!members[m]) continue;
    MemberDev& d = mem_host[m];
    const Problem& Q = *members[m];
    if (d.L == Q.L && d.rho == Q.rho && d.shift == Q.shift) continue;
    d.L = Q.L;
    d.rho = Q.rho;
    d.shift = Q.shift;
    changed = true;
  }
  if (!changed) return;
  // the engine is idle: the table is read by launches queued after this copy (the host image
  // stays unchanged until the copy has run: the next change needs another idle engine, after a
  // synchronisation)
  CGL_HIP(hipMemcpyAsync(memtab.ptr, mem_host, sizeof(mem_host), hipMemcpyHostToDevice, stream));
  CGL_HIP(hipStreamSynchronize(stream));
}

void MixedWork::set_chunk(int c) {
  if (c == chunk) return;
  chunk = c;
  if (graph_exec) {
    CGL_HIP(hipGraphExecDestroy(graph_exec));
    graph_exec = nullptr;
  }
}

int MixedWork::member_of(const Problem* Q) const {
  for (size_t m = 0; m < members.size(); ++m)
    if (members[m] == Q) return (int)m;
  return -1;
}

void MixedWork::forget_member(const Problem* Q) {
  for (auto& m : members)
    if (m == Q) m = nullptr;  // the table entry stays (a slot may still name it until retired)
}

std::vector<int> MixedWork::split_candidates(int64_t m_tiles, int64_t K) {
  std::vector<int> c;
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(16, K / (32 * 16)));
  for (int64_t ks = 1; ks <= cap; ++ks) {
    if (m_tiles * ks > 1024) break;
    const int64_t chunk = round_up((K + ks - 1) / ks, 128);
    if ((K + chunk - 1) / chunk == ks) c.push_back((int)ks);  // distinct chunkings only
  }
  if (c.empty()) c.push_back(1);
  return c;
}

// Every split candidate of the 256-row tiling, then those of the 128-row and the 64-row tilings
// (M rows, a multiple of 256, and a k-length of K).
std::vector<int> MixedWork::tiling_candidates(int64_t M, int64_t K) {
  std::vector<int> c = split_candidates(M / GT_M, K);
  for (int t = 1; t <= 2; ++t)
    for (int ks : split_candidates(M / (GT_M >> t), K)) c.push_back(ks + t * kTile128);
  return c;
}

void MixedWork::set_split_x(int code) {
  const int ks = std::max(1, code_ks(code));
  x_kchunk = round_up((ldp + ks - 1) / ks, 128);
  ksx = (int)((ldp + x_kchunk - 1) / x_kchunk);
  md.ksx = ksx;
  md.x_kchunk = x_kchunk;
  md.x_rt = code_rt(code);
}

void MixedWork::set_split_xt(int code) {
  const int ks = std::max(1, code_ks(code));
  xt_kchunk = round_up((n_pad + ks - 1) / ks, 128);
  ksplit = (int)((n_pad + xt_kchunk - 1) / xt_kchunk);
  md.ksplit = ksplit;
  md.xt_kchunk = xt_kchunk;
  md.xt_rt = code_rt(code);
}

// Autotuner of the tiling of both products (row tile and split-K): every candidate is launched
// on the engine's own buffers (the operands are still zero, the partials are scratch) and timed
// with HIP events.
// Its cost is that time plus the reading of its partial sums by the next kernel (one FP32 slab
// of nodes x rows per chunk, charged at 4 TB/s, about what the consumers achieve); the cheapest
// wins, a later candidate (a larger split, or a shorter row tile) only when it is 2% cheaper.
// Results (the tiling's code) are kept on the context per (pass, rows, k-length, nodes) and in
// the tuning cache file of the device's architecture, which later contexts load
// (CGL_TUNE_CACHE); CGL_AUTOTUNE=0 keeps the 256-row tiling's largest split that fills the chip
// in one round.
void MixedWork::tune_splits(Problem& P) {
  cgl_ctx* ctx = P.ctx;
  hipStream_t s = stream;
  const char* env = std::getenv("CGL_AUTOTUNE");
  const bool tune = !(env && env[0] == '0');
  // test hook: CGL_FORCE_TILE = 256, 128 or 64 keeps only that row tiling (not saved to the
  // cache)
  const char* ft = std::getenv("CGL_FORCE_TILE");
  const int force = ft ? std::atoi(ft) : 0;
  const bool forced = force == 256 || force == 128 || force == 64;
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int> cand = pass == 0 ? split_cands_x : split_cands_xt;
    if (forced) {
      std::vector<int> keep;
      for (int c : cand)
        if (32 * code_rt(c) == force) keep.push_back(c);
      if (!keep.empty()) cand = keep;
    }
    const int64_t m_tiles = pass == 0 ? n_pad / GT_M : ldp / GT_M;
    const std::array<int64_t, 4> key = {pass, pass == 0 ? n_pad : ldp, pass == 0 ? ldp : n_pad,
                                        (int64_t)S_pad};
    auto set = [&](int code) { pass == 0 ? set_split_x(code) : set_split_xt(code); };
    auto launch = [&]() { pass == 0 ? launch_gemm_x(md, s) : launch_gemm_xt(md, s); };
    auto hit = ctx->tuned_split.find(key);
    if (hit != ctx->tuned_split.end() && !forced) {
      set(hit->second);
      ctx->tiling[pass] = hit->second;
      continue;
    }
    int choice = cand.front();
    for (int c : cand)  // without timing: the 256-row tiling's largest split that runs in one round
      if (c < kTile128 && m_tiles * c <= 256) choice = c;
    if (tune && cand.size() > 1) {
      const double slab_ms = (double)S_pad * (pass == 0 ? n_pad : ldp) * 4.0 / 4e12 * 1e3;
      double best = HUGE_VAL;
      for (int code : cand) {
        const int ks = code_ks(code);
        set(code);
        launch();  // warm-up
        CGL_HIP(hipEventRecord(ctx->event(0), s));
        for (int r = 0; r < 3; ++r) launch();
        CGL_HIP(hipEventRecord(ctx->event(1), s));
        CGL_HIP(hipEventSynchronize(ctx->event(1)));
        float ms = 0.f;
        CGL_HIP(hipEventElapsedTime(&ms, ctx->event(0), ctx->event(1)));
        const double cost = ms / 3.0 + ks * slab_ms;
        if (cost < best * 0.98) {
          best = cost;
          choice = code;
        }
      }
    }
    set(choice);
    ctx->tiling[pass] = choice;
    if (forced) continue;
    ctx->tuned_split[key] = choice;
    if (tune && cand.size() > 1) ctx->save_tuning(key, choice);
  }
}

// One iteration of Alg. 3 for every running slot; ev (optional): events around the two MFMA
// passes for kernel timing.
// ev: events that the product launches update with their start and end (ev[2], ev[3]: X^T pass;
// ev[0], ev[1]: X pass, with time_x). A timed launch still starts a few microseconds later than
// an untimed one, so the X pass is timed only when asked.
static void mixed_cycle(MixedWork& W, hipStream_t s, hipEvent_t* ev = nullptr, bool time_x = false) {
  const bool tx = ev != nullptr && time_x;
  launch_gemm_x(W.md, s, true, tx ? ev[0] : nullptr, tx ? ev[1] : nullptr);
  launch_mixed_loss(W.md, s);
  launch_mixed_decide(W.md, s);
  launch_gemm_xt(W.md, s, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
  launch_mixed_node(W.md, s);
}

static bool mixed_graphs() {
  const char* e = std::getenv("CGL_NO_GRAPH");
  return !(e && e[0] == '1');
}

void MixedWork::reorder_probe(Problem& P) {
  // the counts reach the host with the chunk's state copy (the control tail of st)
  hipStream_t s = stream;
  launch_perm_flags(md, sflag.as<uint8_t>(), s);
  launch_perm_build(sflag.as<uint8_t>(), P.p, ldp, perm_new.as<int>(), pinv_new.as<int>(),
                    ctl_dev() + kCtlUnion, s);
}

void MixedWork::reorder_apply(Problem& P) {
  hipStream_t s = stream;
  const int* h = ctl_host();
  const int64_t grain = 2 * GT_K;
  const int64_t now = round_up(std::max(h[kCtlExtent], h[kCtlExtent + 1]), grain);
  int64_t after = std::min(round_up(h[kCtlUnion], grain), ldp);
  if (prefix_cap > 0) after = std::min(after, prefix_cap);
  int64_t strays = 0;
  for (int i = 0; i < S; ++i) strays += h[kCtlStrays + i];
  // a stray costs its slot a column of X~ every cycle (one row of X~^T read by the loss kernel);
  // a reorder rewrites X~ once (about 0.25 ms)
  const bool shorter = after <= now - std::max<int64_t>(2 * grain, now / reorder_shrink);
  if (!shorter && strays <= S) return;  // the current order still serves
  CGL_HIP(hipMemcpyAsync(dop_tmp.ptr, dop.ptr, dop.bytes, hipMemcpyDeviceToDevice, s));
  CGL_HIP(hipMemsetAsync(md.keff, 0, 2 * sizeof(int), s));  // the extent counters only
  launch_perm_operand(md, dop_tmp.as<uint16_t>(), pinv.as<int>(), pinv_new.as<int>(), s);
  launch_perm_design(Xbt.as<uint16_t>(), n_pad, perm_new.as<int>(), P.p, Xb.as<uint16_t>(), ldp,
                     s);
  CGL_HIP(hipMemcpyAsync(pinv.ptr, pinv_new.ptr, (size_t)ldp * sizeof(int),
                         hipMemcpyDeviceToDevice, s));
  CGL_HIP(hipMemcpyAsync(perm.ptr, perm_new.ptr, (size_t)ldp * sizeof(int),
                         hipMemcpyDeviceToDevice, s));
  // the union fills the prefix; later entrants behind it become strays (the staging value is
  // rewritten only after the next chunk's synchronisation, when this copy has run)
  *order_host = (int)after;
  CGL_HIP(hipMemcpyAsync(pfx.ptr, order_host, sizeof(int), hipMemcpyHostToDevice, s));
  reorders += 1;
  if (P.ctx->profiling || P.ctx->phase_timing) P.ctx->kt_n[12] += 1;
}

void MixedWork::launch_chunk(Problem& P) {
  hipStream_t s = stream;
  cgl_ctx* ctx = P.ctx;
  // with profiling on, each cycle's X^T pass (and at level 2 its X pass) is bracketed by HIP
  // events on the stream (HIP cannot time events recorded inside a graph, so the cycles are then
  // launched one by one)
  if (ctx->profiling || !mixed_graphs()) {
    for (int i = 0; i < chunk; ++i) {
      hipEvent_t ev[4];
      for (int e = 0; e < 4; ++e) ev[e] = ctx->event((size_t)(4 * i + e));
      mixed_cycle(*this, s, ctx->profiling ? ev : nullptr, ctx->profile_x);
    }
  } else {
    if (!graph_exec) {
      hipGraph_t graph;
      CGL_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < chunk; ++i) mixed_cycle(*this, s);
      CGL_HIP(hipStreamEndCapture(s, &graph));
      CGL_HIP(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
      CGL_HIP(hipGraphDestroy(graph));
    }
    // level 3: the GPU span of the chunk (launch gaps inside the graph included)
    if (ctx->phase_timing) CGL_HIP(hipEventRecord(ctx->event(200), s));
    CGL_HIP(hipGraphLaunch(graph_exec, s));
    if (ctx->phase_timing) CGL_HIP(hipEventRecord(ctx->event(201), s));
  }
  // the operand order is checked with the chunk's own synchronisation and changed (if at all)
  // before the next launches
  chunk_probe = reorder && cycles + chunk - reorder_checked >= reorder_every;
  if (chunk_probe) reorder_probe(P);
  // iterates retired before this chunk go to the callers' buffers while the chunk runs
  flush_retired();
  CGL_HIP(hipMemcpyAsync(st_host, st.ptr, st_bytes(), hipMemcpyDeviceToHost, s));
  CGL_HIP(hipEventRecord(chunk_done, s));
  in_flight = true;
}

void MixedWork::finish_chunk(Problem& P) {
  cgl_ctx* ctx = P.ctx;
  in_flight = false;
  close_round(P);  // a certification round queued before this chunk has finished too
  // X-pass extent statistics (cumulative on the device): this chunk's share
  const int* h = ctl_host();
  const int es[2] = {h[kCtlExtent + 2] - ext_seen[0], h[kCtlExtent + 3] - ext_seen[1]};
  ext_seen[0] = h[kCtlExtent + 2];
  ext_seen[1] = h[kCtlExtent + 3];
  if (chunk_probe) {
    reorder_checked = cycles + chunk;
    reorder_apply(P);
  }
  if (ctx->profiling || ctx->phase_timing) {
    // mean X-pass operand extent: total = sum of the extents as fractions of ldp, count = passes
    ctx->kt_ms[9] += (double)es[0] * (2 * GT_K) / (double)ldp;
    ctx->kt_n[9] += es[1];
  }
  if (ctx->profiling) {
    for (int i = 0; i < chunk; ++i) {
      float a = 0.f, b = 0.f;
      if (ctx->profile_x) {
        CGL_HIP(hipEventElapsedTime(&a, ctx->event((size_t)(4 * i)), ctx->event((size_t)(4 * i + 1))));
        ctx->kt_ms[3] += a;  // X pass
        ctx->kt_n[3] += 1;
      }
      CGL_HIP(hipEventElapsedTime(&b, ctx->event((size_t)(4 * i + 2)), ctx->event((size_t)(4 * i + 3))));
      ctx->kt_ms[2] += b;  // X^T pass
      ctx->kt_n[2] += 1;
    }
  }
  if (ctx->phase_timing && !ctx->profiling && mixed_graphs()) {
    float a = 0.f;
    CGL_HIP(hipEventElapsedTime(&a, ctx->event(200), ctx->event(201)));
    ctx->kt_ms[10] += a;
    ctx->kt_n[10] += 1;
  }
  cycles += chunk;
}

// Waits for an event by polling it: the host takes up the chunk's outcome within microseconds
// of the GPU reaching the event (a blocking wait returns later, and the GPU idles meanwhile).
static void poll_event(hipEvent_t e) {
  static const bool block = [] {
    const char* v = std::getenv("CGL_BLOCKING_WAIT");
    return v && std::atoi(v) > 0;
  }();
  if (block) {
    CGL_HIP(hipEventSynchronize(e));
    return;
  }
  for (;;) {
    const hipError_t r = hipEventQuery(e);
    if (r == hipSuccess) return;
    if (r != hipErrorNotReady) CGL_HIP(r);
  }
}

void MixedWork::run_chunk(Problem& P) {
  launch_chunk(P);
  poll_event(chunk_done);
  finish_chunk(P);
}

int MixedWork::cert_round(Problem& P, bool overlap) {
  // Batch the FP64 rounds: a node that asks for certification keeps iterating until enough
  // nodes ask (cert_batch), the oldest request has waited cert_wait chunks, or every active node
  // is waiting, so each round's FP64 products are shared by more nodes.
  std::vector<int> want;
  int active = 0;
  int64_t oldest = cycles;
  for (int sl = 0; sl < S; ++sl) {
    const NodeDev& d = st_host[sl];
    if (slot_owner[(size_t)sl] < 0 || !d.active || d.done) {
      want_since[sl] = -1;
      continue;
    }
    ++active;
    if (!d.want_cert) {
      want_since[sl] = -1;
      continue;
    }
    if (want_since[sl] < 0) want_since[sl] = cycles;
    oldest = std::min(oldest, want_since[sl]);
    want.push_back(sl);
  }
  if (want.empty()) return kRoundNone;
  const int nq = (int)want.size();
  bool parked = false;  // a warm start waiting for its base point cannot wait for others
  for (int sl : want) parked = parked || st_host[sl].need_base;
  if (!parked && nq < cert_batch && nq < active && cycles - oldest < (int64_t)cert_wait * chunk)
    return kRoundNone;
  // left open when other nodes keep running: the next chunk is queued behind the round and its
  // synchronisation brings the round's outcome too
  overlap = overlap && nq < active;
  hipStream_t s = stream;
  cgl_ctx* ctx = P.ctx;
  for (int sl : want) want_since[sl] = -1;
  // least-squares nodes first: with a Gram matrix they take its rows (the first nls of the list)
  // and only the others the FP64 product with all of X^T
  int nls = 0;
  if (G.ptr != nullptr) {
    std::stable_partition(want.begin(), want.end(), [&](int sl) {
      return mem_host[st_host[sl].member].loss == LOSS_LS;
    });
    for (int sl : want) nls += mem_host[st_host[sl].member].loss == LOSS_LS ? 1 : 0;
  }
  upload_list(P, want, kListCert);
  hipEvent_t e0 = ctx->profiling ? ctx->event(100) : nullptr;
  hipEvent_t e1 = ctx->profiling ? ctx->event(101) : nullptr;
  const bool span = ctx->phase_timing && !ctx->profiling;  // level 3: the round's GPU span
  if (span) CGL_HIP(hipEventRecord(ctx->event(202), s));
  // X beta in FP64 over the union of the iterates' supports (the other coordinates contribute
  // exact zeros), from the rows of the transposed design
  launch_cert_gather(md, list.as<int>(), nq, B64.as<double>(), sflag.as<uint8_t>(), s);
  launch_cert_support(sflag.as<uint8_t>(), P.p, sidx.as<int>(), scount.as<int>(), s);
  // the union's size stays on the device: the products read it at launch and split it over
  // chunks sized for all p coordinates
  CGL_HIP(hipMemcpyAsync(count_host, scount.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  const void* xt = P.xtype == XT_BF16 ? Xbt.ptr : Xt.ptr;
  const int* kdev = scount.as<int>();
  if (e0) CGL_HIP(hipEventRecord(e0, s));
  launch_cert_compact(B64.as<double>(), ldp, sidx.as<int>(), kdev, P.p, nq, Bu.as<double>(), s);
  launch_gemm_f64_rows(P.xtype, xt, n_pad, sidx.as<int>(), P.n, P.p, kdev, Bu.as<double>(), ldp,
                       nq, U64.as<double>(), n_pad, part64.as<double>(), part64_cap, s);
  if (e1) CGL_HIP(hipEventRecord(e1, s));
  // X^T grad f(X beta): the least-squares nodes from the Gram rows on the same support (p K
  // against n p products), the others by the FP64 product with all of X^T
  if (nls > 0) {
    launch_gemm_f64_rows(XT_F64, G.ptr, ldg, sidx.as<int>(), P.p, P.p, kdev, Bu.as<double>(), ldp,
                         nls, H64.as<double>(), ldp, part64.as<double>(), part64_cap, s);
    launch_gram_finish(H64.as<double>(), ldp, P.p, nls, md, list.as<int>(), s);
  }
  launch_cert_resid(md, list.as<int>(), nq, U64.as<double>(), R64.as<double>(),
                    cpart.as<double>(), ncchunk, cchunk, s);
  if (nls < nq)
    launch_gemm_f64(P.xtype, xt, n_pad, P.p, P.n, R64.as<double>() + (int64_t)nls * n_pad, n_pad,
                    nq - nls, H64.as<double>() + (int64_t)nls * ldp, ldp, part64.as<double>(),
                    part64_cap, s);
  launch_cert_finish(md, list.as<int>(), nq, B64.as<double>(), H64.as<double>(),
                     cpart.as<double>(), ncchunk, s);
  if (span) CGL_HIP(hipEventRecord(ctx->event(203), s));
  round_span = span;
  round_open = true;
  if (overlap) return kRoundOpen;
  CGL_HIP(hipMemcpyAsync(st_host, st.ptr, (size_t)S * sizeof(NodeDev), hipMemcpyDeviceToHost, s));
  CGL_HIP(hipStreamSynchronize(s));
  close_round(P);
  return kRoundDone;
}

void MixedWork::close_round(Problem& P) {
  if (!round_open) return;
  round_open = false;
  if (*count_host < 0 || *count_host > P.p) throw std::runtime_error("support union out of range");
  support_sum += *count_host;
  cgl_ctx* ctx = P.ctx;
  if (ctx->profiling) {
    float a = 0.f;
    CGL_HIP(hipEventElapsedTime(&a, ctx->event(100), ctx->event(101)));
    ctx->kt_ms[4] += a;
    ctx->kt_n[4] += 1;
  }
  if (round_span) {
    float a = 0.f;
    CGL_HIP(hipEventElapsedTime(&a, ctx->event(202), ctx->event(203)));
    ctx->kt_ms[11] += a;
    ctx->kt_n[11] += 1;
    round_span = false;
  }
  cert_rounds += 1;
}

size_t MixedWork::device_bytes() const {
  const DevBuf* bufs[] = {&Xb, &Xbt, &memtab, &st, &cls, &bring, &beta0, &H0, &base0, &base1, &e0f,
                          &bres, &bdual, &dop, &gop, &gop_r, &gsel, &dU, &dUp, &dH, &lpart, &npart, &fpart, &cycle, &prevsel, &B64,
                          &U64, &R64, &H64, &cpart, &list,
                          &Xt, &part64, &sflag, &sidx, &scount, &Bu, &G, &pinv, &pinv_new,
                          &perm, &perm_new, &dop_tmp, &pfx, &sj, &sv, &Bret};
  size_t b = 0;
  for (const DevBuf* d : bufs) b += d->bytes;
  for (const auto& m : mbufs) b += m->y.bytes + m->H0c.bytes + m->b0c.bytes + m->b1c.bytes;
  return b;
}

int MixedWork::free_slots() const {
  int c = 0;
  for (int o : slot_owner) c += o < 0 ? 1 : 0;
  return c;
}

void MixedWork::admit(Problem& P, const std::vector<Admission>& adm) {
  if (adm.empty()) return;
  hipStream_t s = stream;
  std::vector<int> slots;
  for (const Admission& a : adm) {
    const int sl = a.slot;
    slots.push_back(sl);
    slot_owner[(size_t)sl] = a.owner;
    NodeDev d = make_node_dev(a.node, a.host);
    d.member = a.member;
    d.active = 1;
    d.primed = 0;
    d.P_best = HUGE_VAL;
    d.D_best = -HUGE_VAL;
    d.P_cert = HUGE_VAL;
    d.D_cert = -HUGE_VAL;
    d.mgap_ref = HUGE_VAL;
    d.L_prev = HUGE_VAL;
    d.g_new = 0.0;  // g(0)
    if (d.iter >= d.max_iter) d.want_cert = 1;  // no iteration allowed: certify the start
    if (a.node.warm_start) {
      // parked until the next FP64 round evaluates the bound at the start and moves the base
      // point there; its g is not evaluated, so the start never counts as a best primal value
      d.need_base = 1;
      d.want_cert = 1;
      d.g_new = HUGE_VAL;
    }
    st_host[sl] = d;
    std::copy(a.host.cls.begin(), a.host.cls.end(), cls_host + (int64_t)sl * ldp);
    std::fill(cls_host + (int64_t)sl * ldp + P.p, cls_host + (int64_t)(sl + 1) * ldp,
              (uint8_t)CLS_PAD);
    admitted_at[sl] = cycles;
  }
  upload_list(P, slots, kListAdmit);
  // the admitted slots' class rows and states, one copy per run of consecutive slots (the other
  // slots' device states stay as they are: a certification round queued earlier may still be
  // writing them); the cold-start kernel then reads each slot's problem from its state
  {
    std::vector<int> ss = slots;
    std::sort(ss.begin(), ss.end());
    for (size_t a = 0; a < ss.size();) {
      size_t b = a + 1;
      while (b < ss.size() && ss[b] == ss[b - 1] + 1) ++b;
      const size_t off = (size_t)ss[a] * ldp, len = (b - a) * (size_t)ldp;
      CGL_HIP(hipMemcpyAsync((uint8_t*)cls.ptr + off, cls_host + off, len, hipMemcpyHostToDevice, s));
      CGL_HIP(hipMemcpyAsync(st.as<NodeDev>() + ss[a], st_host + ss[a], (b - a) * sizeof(NodeDev),
                             hipMemcpyHostToDevice, s));
      a = b;
    }
  }
  launch_admit(md, list.as<int>(), (int)slots.size(), s);
  if (P.ctx->profiling || P.ctx->phase_timing) P.ctx->kt_n[13] += (int64_t)slots.size();
  // warm starts (fixed-zero coordinates set to 0) into the iterate ring, the base and the best
  std::vector<std::vector<double>> starts;
  for (const Admission& a : adm) {
    if (!a.node.warm_start) continue;
    starts.emplace_back(a.node.warm_start, a.node.warm_start + P.p);
    std::vector<double>& ws = starts.back();
    for (int64_t j = 0; j < P.p; ++j)
      if (a.host.cls[(size_t)j] == CLS_ZERO) ws[(size_t)j] = 0.0;
    const int64_t o = (int64_t)a.slot * ldp;
    for (int r = 0; r < 3; ++r)
      CGL_HIP(hipMemcpyAsync(bring.as<double>() + (int64_t)r * S * ldp + o, ws.data(),
                             (size_t)P.p * 8, hipMemcpyHostToDevice, s));
    CGL_HIP(hipMemcpyAsync(beta0.as<double>() + o, ws.data(), (size_t)P.p * 8,
                           hipMemcpyHostToDevice, s));
    CGL_HIP(hipMemcpyAsync(bres.as<double>() + o, ws.data(), (size_t)P.p * 8,
                           hipMemcpyHostToDevice, s));
  }
  // The staged warm starts are local: their copies must finish before they go. The other
  // staging (slot states, class rows, the list) is pinned and rewritten only after the next
  // chunk's event, and the stream orders these copies before that chunk, so the host need not
  // wait for them (nor for a certification round queued ahead of them).
  if (!starts.empty()) CGL_HIP(hipStreamSynchronize(s));
  if (reorder && (int)adm.size() >= S / 4) {
    // many new supports: no prefix (no strays) until a check half an interval later lists them
    const int nopfx = (int)ldp;
    CGL_HIP(hipMemcpy(pfx.ptr, &nopfx, sizeof(int), hipMemcpyHostToDevice));
    reorder_checked = cycles - kReorderEvery / 2;
  }
}

void MixedWork::retire(Problem& P, const std::vector<int>& slots,
                       const std::vector<cgl_result*>& res, const std::vector<double*>& beta_out,
                       bool defer, const std::vector<double*>* dual_out) {
  hipStream_t s = stream;
  if (dual_out) {
    for (size_t i = 0; i < slots.size(); ++i)
      if ((*dual_out)[i])
        CGL_HIP(hipMemcpyAsync((*dual_out)[i], bdual.as<double>() + (int64_t)slots[i] * ldp,
                               (size_t)P.p * 8, hipMemcpyDeviceToHost, s));
    CGL_HIP(hipStreamSynchronize(s));
  }
  std::vector<int> rows;  // slots whose iterate is wanted, in the order of their staging rows
  for (size_t i = 0; i < slots.size(); ++i) {
    const int sl = slots[i];
    const NodeDev& d = st_host[sl];
    cgl_result* r = res[i];
    r->primal = d.P_cert;
    r->lower_bound = d.D_cert;
    r->gap_abs = d.P_cert - d.D_cert;
    r->gap_rel = r->gap_abs / std::max(std::fabs(d.P_cert), 1.0);
    r->iters = d.iter - 1;
    r->restarts = d.restarts;
    r->status = d.status == kRunning ? CGL_NOT_CONVERGED : d.status;
    r->recentres = d.recentres;
    r->err_vs_fp64_est = std::isfinite(d.P_cert)
                             ? std::fabs(d.L_work - d.P_cert) / std::max(std::fabs(d.P_cert), 1.0)
                             : 0.0;
    if (beta_out[i]) rows.push_back(sl);
  }
  if (!rows.empty()) {
    flush_retired();  // the staging rows of the previous retirement are free again
    const int nq = (int)rows.size();
    upload_list(P, rows, kListRetire);
    // the gather overwrites Bret: the previous deferred copy must have read it
    if (ret_copy_recorded) CGL_HIP(hipStreamWaitEvent(s, ret_copied, 0));
    launch_gather_rows(bres.as<double>(), ldp, list.as<int>(), nq, P.p, Bret.as<double>(), s);
    const size_t bytes = (size_t)nq * P.p * sizeof(double);
    for (size_t i = 0; i < slots.size(); ++i)
      if (beta_out[i]) ret_pending.push_back(beta_out[i]);
    if (defer) {
      CGL_HIP(hipEventRecord(ret_gathered, s));
      CGL_HIP(hipStreamWaitEvent(copy_stream, ret_gathered, 0));
      CGL_HIP(hipMemcpyAsync(beta_host, Bret.ptr, bytes, hipMemcpyDeviceToHost, copy_stream));
      CGL_HIP(hipEventRecord(ret_copied, copy_stream));
      ret_copy_recorded = true;
    } else {
      CGL_HIP(hipMemcpyAsync(beta_host, Bret.ptr, bytes, hipMemcpyDeviceToHost, s));
      CGL_HIP(hipStreamSynchronize(s));
      ret_copy_recorded = false;
    }
    pending_p = P.p;
    if (!defer) flush_retired();
  }
  for (int sl : slots) {
    st_host[sl].active = 0;
    slot_owner[(size_t)sl] = -1;
  }
}

// A slot list to the device (list), through the pinned region of its caller.
void MixedWork::upload_list(Problem& P, const std::vector<int>& v, int region) {
  int* h = list_host + (size_t)region * S;
  std::copy(v.begin(), v.end(), h);
  CGL_HIP(hipMemcpyAsync(list.ptr, h, v.size() * sizeof(int), hipMemcpyHostToDevice,
                         stream));
}

void MixedWork::drop_retired() {
  if (ret_copy_recorded) CGL_HIP(hipEventSynchronize(ret_copied));
  ret_pending.clear();
}

void MixedWork::flush_retired() {
  if (ret_pending.empty()) return;
  if (ret_copy_recorded) CGL_HIP(hipEventSynchronize(ret_copied));
  for (size_t q = 0; q < ret_pending.size(); ++q)
    std::memcpy(ret_pending[q], beta_host + q * pending_p, (size_t)pending_p * sizeof(double));
  ret_pending.clear();
}

// Upload the host image of all slot states (after retire/admit edits; nothing of the engine is
// in flight).
void MixedWork::push_states(Problem& P) {
  CGL_HIP(hipMemcpyAsync(st.ptr, st_host, (size_t)S * sizeof(NodeDev), hipMemcpyHostToDevice,
                         stream));
}

void solve_mixed(Problem& Pm, const cgl_node* nodes, int32_t count, double* beta_out,
                 cgl_result* res, const int32_t* rows, double* dual_out) {
  // node i reports into the caller's row rows[i] (res and beta_out), or row i
  auto row = [&](int32_t i) -> int64_t { return rows ? rows[i] : i; };
  // the nodes are Pm's; the engine is that of the problem owning Pm's design (Pm itself unless
  // Pm shares another problem's design)
  Problem& P = Pm.engine_problem();
  if (!P.mixed) P.mixed = new MixedWork();
  MixedWork& W = *P.mixed;
  W.ensure(P);
  const int member = W.member_of(&Pm);
  if (member < 0) invalid("the problem's design was shared after its owner's engine was built");
  if (W.free_slots() != W.S)
    invalid("the problem's batched engine is in use by a server; solve through the server");
  if (Pm.shift != 0.0 && Pm.loss != LOSS_LS)
    invalid("the eigen-perspective relaxation is for least squares");
  if (W.in_flight) invalid("the problem's batched engine is in use by a server");
  W.set_relaxation(P);
  W.set_chunk(W.solve_chunk);
  W.stream = P.ctx->stream;  // a server may have run it on a stream of its own
  hipStream_t s = W.stream;
  // a solve that failed part-way may have left staged iterates for buffers that are gone
  W.drop_retired();
  std::vector<NodeHost> hosts;
  hosts.reserve((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    hosts.push_back(make_node_host(nodes[i], P.p, Pm.k));
  }
  int32_t next = 0, finished = 0;
  // infeasible nodes never take a slot
  std::vector<char> handled((size_t)count, 0);
  for (int32_t i = 0; i < count; ++i) {
    if (hosts[(size_t)i].infeasible) {
      infeasible_result(&res[row(i)], beta_out ? beta_out + row(i) * P.p : nullptr, P.p);
      handled[(size_t)i] = 1;
      ++finished;
    }
  }
  auto fill = [&]() {
    std::vector<Admission> adm;
    for (int sl = 0; sl < W.S && next < count; ++sl) {
      if (W.slot_owner[(size_t)sl] >= 0) continue;
      while (next < count && handled[(size_t)next]) ++next;
      if (next >= count) break;
      adm.push_back(Admission{sl, next, nodes[next], hosts[(size_t)next], member});
      ++next;
    }
    W.admit(P, adm);
  };
  cgl_ctx* ctx = P.ctx;
  auto phase = [&](int which, auto&& fn) {
    if (!ctx->phase_timing) return fn();
    const auto t0 = std::chrono::steady_clock::now();
    fn();
    ctx->kt_ms[which] +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ctx->kt_n[which] += 1;
  };
  phase(7, [&] { fill(); });
  phase(5, [&] { W.run_chunk(P); });
  while (finished < count) {
    // A round left open runs ahead of the next chunk and shares its synchronisation; the
    // retirements of nodes certified by earlier rounds (and the admissions into their slots)
    // are queued behind it, so the host's part of them overlaps the round's device work. A
    // closed round (no other node running) has synchronised, and its nodes retire at once.
    phase(6, [&] { (void)W.cert_round(P, /*overlap=*/true); });
    phase(7, [&] {
      std::vector<int> done;
      std::vector<cgl_result*> rs;
      std::vector<double*> bs, ds;
      for (int sl = 0; sl < W.S; ++sl) {
        const int owner = W.slot_owner[(size_t)sl];
        if (owner < 0 || !W.st_host[sl].done) continue;
        done.push_back(sl);
        rs.push_back(&res[row(owner)]);
        bs.push_back(beta_out ? beta_out + row(owner) * P.p : nullptr);
        ds.push_back(dual_out ? dual_out + row(owner) * P.p : nullptr);
      }
      if (!done.empty()) {
        W.retire(P, done, rs, bs, /*defer=*/true, dual_out ? &ds : nullptr);
        finished += (int32_t)done.size();
        // the device states of the retired slots need no update: they are done and do not run,
        // and an admission into the slot writes its state
        fill();
      }
    });
    // a run with nothing active and work pending would spin: guard
    if (finished < count && W.free_slots() == W.S && next >= count) break;
    if (finished < count) phase(5, [&] { W.run_chunk(P); });
  }
  CGL_HIP(hipStreamSynchronize(s));
  W.flush_retired();
}

}  // namespace cgl

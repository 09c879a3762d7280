// Request server: continuous batching of node relaxations over resident problems.
//
// Submitted nodes wait in a FIFO queue. Each poll runs one scheduling round:
//   1. admission: queued mixed-precision nodes take free device slots of their problem's batched
//      engine (at most max_slots per problem); a problem whose engine is not resident yet is
//      brought in only while the device memory of all resident engines stays within the budget
//      (an idle engine is released when another problem needs the room);
//   2. one FP64-path node (precision F64) is solved to completion, if one is queued;
//   3. every engine with running slots advances one chunk of iterations and its certification
//      round; finished, cancelled or certified slots are retired and refilled on the next round.
// Results wait in a completion list until polled. Everything runs on the context's stream from
// the calling thread; calls on one server must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <memory>
#include <vector>

#include "batch.h"
#include "common.h"
#include "engine.h"

namespace cgl {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket = 0;
  Problem* P = nullptr;
  cgl_node node{};
  std::vector<int32_t> z0, z1;
  std::vector<double> warm;
  NodeHost host;
  double t_submit = 0.0;
  bool cancelled = false;
};

struct Finished {
  uint64_t ticket = 0;
  cgl_result res{};
  std::vector<double> beta;
  double latency = 0.0;
};

// A problem whose batched engine is resident, with the request held by each of its slots.
struct Resident {
  Problem* P = nullptr;
  std::vector<std::unique_ptr<Request>> slot_req;  // kSlots entries
  int running() const {
    int c = 0;
    for (const auto& r : slot_req) c += r ? 1 : 0;
    return c;
  }
};

constexpr size_t kQueueCap = 1u << 20;

}  // namespace

}  // namespace cgl

struct cgl_server {
  cgl_ctx* ctx = nullptr;
  size_t budget = 0;  // 0: no limit
  int max_slots = cgl::kSlots;
  uint64_t next_ticket = 1;
  std::deque<std::unique_ptr<cgl::Request>> queue;
  std::vector<cgl::Resident> resident;
  std::deque<cgl::Finished> done;
};

namespace cgl {

namespace {

void finish(cgl_server& S, std::unique_ptr<Request> r, const cgl_result& res,
            std::vector<double> beta) {
  Finished f;
  f.ticket = r->ticket;
  f.res = res;
  f.beta = std::move(beta);
  f.latency = now_s() - r->t_submit;
  S.done.push_back(std::move(f));
}

Resident* find_resident(cgl_server& S, Problem* P) {
  for (auto& R : S.resident)
    if (R.P == P) return &R;
  return nullptr;
}

size_t resident_bytes(const cgl_server& S) {
  size_t b = 0;
  for (const auto& R : S.resident) b += R.P->mixed ? R.P->mixed->device_bytes() : 0;
  return b;
}

bool has_queued(const cgl_server& S, const Problem* P) {
  for (const auto& r : S.queue)
    if (r->P == P && r->node.precision == CGL_PREC_MIXED) return true;
  return false;
}

// Bring P's batched engine in, releasing idle engines of other problems if the budget needs it.
// A single engine is always admitted when nothing else is resident (the budget caps co-residency).
Resident* make_resident(cgl_server& S, Problem* P) {
  if (Resident* R = find_resident(S, P)) return R;
  if (S.budget > 0) {
    // release idle engines (no running slot, nothing queued)
    for (size_t i = 0; i < S.resident.size();) {
      Resident& R = S.resident[i];
      if (R.running() == 0 && !has_queued(S, R.P)) {
        delete R.P->mixed;
        R.P->mixed = nullptr;
        S.resident.erase(S.resident.begin() + (ptrdiff_t)i);
      } else {
        ++i;
      }
    }
    const size_t busy = resident_bytes(S);
    if (P->mixed_bytes > 0 && busy + P->mixed_bytes > S.budget && !S.resident.empty())
      return nullptr;  // wait for the busy engines to drain
  }
  if (!P->mixed) P->mixed = new MixedWork();
  P->mixed->ensure(*P);
  P->mixed_bytes = P->mixed->device_bytes();
  if (S.budget > 0 && !S.resident.empty() &&
      resident_bytes(S) + P->mixed_bytes > S.budget) {
    // footprint learnt just now and it does not fit beside the busy engines
    delete P->mixed;
    P->mixed = nullptr;
    return nullptr;
  }
  Resident R;
  R.P = P;
  R.slot_req.resize((size_t)P->mixed->S);
  S.resident.push_back(std::move(R));
  return &S.resident.back();
}

void admit_round(cgl_server& S) {
  // reserve slots in queue order, then admit per problem in one call each
  std::vector<Problem*> blocked;
  std::vector<std::pair<Problem*, std::vector<Admission>>> batches;
  for (auto it = S.queue.begin(); it != S.queue.end();) {
    Request& q = **it;
    if (q.node.precision != CGL_PREC_MIXED ||
        std::find(blocked.begin(), blocked.end(), q.P) != blocked.end()) {
      ++it;
      continue;
    }
    Resident* R = make_resident(S, q.P);
    int slot = -1;
    if (R && R->running() < S.max_slots) {
      const MixedWork& W = *q.P->mixed;
      for (int sl = 0; sl < W.S; ++sl)
        if (W.slot_owner[(size_t)sl] < 0 && !R->slot_req[(size_t)sl]) { slot = sl; break; }
    }
    if (slot < 0) {
      blocked.push_back(q.P);
      ++it;
      continue;
    }
    auto bt = std::find_if(batches.begin(), batches.end(),
                           [&](const auto& b) { return b.first == q.P; });
    if (bt == batches.end()) {
      batches.emplace_back(q.P, std::vector<Admission>());
      bt = batches.end() - 1;
    }
    bt->second.push_back(Admission{slot, slot, q.node, q.host});
    R->slot_req[(size_t)slot] = std::move(*it);
    it = S.queue.erase(it);
  }
  for (auto& b : batches) b.first->mixed->admit(*b.first, b.second);
}

void plain_round(cgl_server& S) {
  for (auto it = S.queue.begin(); it != S.queue.end(); ++it) {
    if ((*it)->node.precision == CGL_PREC_MIXED) continue;
    std::unique_ptr<Request> r = std::move(*it);
    S.queue.erase(it);
    cgl_result res{};
    std::vector<double> beta((size_t)r->P->p);
    solve_plain(*r->P, r->node, r->host, beta.data(), &res);
    finish(S, std::move(r), res, std::move(beta));
    return;  // one per round keeps the batched slots moving
  }
}

void run_round(cgl_server& S) {
  for (auto& R : S.resident) {
    if (R.running() == 0) continue;
    Problem& P = *R.P;
    MixedWork& W = *P.mixed;
    W.run_chunk(P);
    W.cert_round(P);
    std::vector<int> done;
    for (int sl = 0; sl < W.S; ++sl) {
      const std::unique_ptr<Request>& r = R.slot_req[(size_t)sl];
      if (r && (W.st_host[sl].done || r->cancelled)) done.push_back(sl);
    }
    if (!done.empty()) {
      std::vector<cgl_result> res(done.size());
      std::vector<std::vector<double>> betas(done.size(), std::vector<double>((size_t)P.p));
      std::vector<cgl_result*> rs;
      std::vector<double*> bs;
      for (size_t i = 0; i < done.size(); ++i) {
        rs.push_back(&res[i]);
        bs.push_back(betas[i].data());
      }
      W.retire(P, done, rs, bs);
      for (size_t i = 0; i < done.size(); ++i) {
        std::unique_ptr<Request>& r = R.slot_req[(size_t)done[i]];
        if (r->cancelled) res[i].status = CGL_CANCELLED;
        finish(S, std::move(r), res[i], std::move(betas[i]));
      }
      W.push_states(P);
      CGL_HIP(hipStreamSynchronize(P.ctx->stream));
    }
  }
}

}  // namespace

}  // namespace cgl

using namespace cgl;

extern "C" {

int cgl_server_create(cgl_ctx* ctx, size_t hbm_budget_bytes, int32_t max_slots,
                      cgl_server** out) {
  CGL_API_BEGIN
  if (!out) invalid("out is NULL");
  *out = nullptr;
  if (!ctx) invalid("ctx is NULL");
  if (max_slots < 1 || max_slots > kSlots) invalid("max_slots must be in [1, 256]");
  std::unique_ptr<cgl_server> s(new cgl_server());
  s->ctx = ctx;
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  *out = s.release();
  return CGL_OK;
  CGL_API_END
}

int cgl_server_submit(cgl_server* srv, cgl_problem* prob, const cgl_node* node,
                      uint64_t* ticket) {
  CGL_API_BEGIN
  if (!srv || !prob || !node || !ticket) invalid("NULL argument");
  Problem* P = reinterpret_cast<Problem*>(prob);
  if (P->ctx != srv->ctx) invalid("the problem belongs to another context");
  if (P->shift != 0.0 && node->precision == CGL_PREC_MIXED)
    invalid("the eigen-perspective relaxation runs on the FP64 path (CGL_PREC_F64)");
  if (srv->queue.size() >= kQueueCap) {
    set_error("server queue is full");
    return CGL_E_BUSY;
  }
  std::unique_ptr<Request> r(new Request());
  r->host = make_node_host(*node, P->p, P->k);  // validates
  r->ticket = srv->next_ticket++;
  r->P = P;
  r->node = *node;
  r->z0.assign(node->fixed_zero, node->fixed_zero + node->n_zero);
  r->z1.assign(node->fixed_in, node->fixed_in + node->n_in);
  r->node.fixed_zero = r->z0.empty() ? nullptr : r->z0.data();
  r->node.fixed_in = r->z1.empty() ? nullptr : r->z1.data();
  if (node->warm_start) {
    r->warm.assign(node->warm_start, node->warm_start + P->p);
    r->node.warm_start = r->warm.data();
  }
  r->t_submit = now_s();
  *ticket = r->ticket;
  if (r->host.infeasible) {
    cgl_result res{};
    std::vector<double> beta((size_t)P->p);
    infeasible_result(&res, beta.data(), P->p);
    finish(*srv, std::move(r), res, std::move(beta));
  } else {
    srv->queue.push_back(std::move(r));
  }
  return CGL_OK;
  CGL_API_END
}

int cgl_server_poll(cgl_server* srv, int32_t max, uint64_t* tickets, cgl_result* res,
                    double* betas, int64_t betas_stride, double* latency_s, int32_t* got) {
  CGL_API_BEGIN
  if (!srv || !got) invalid("NULL argument");
  *got = 0;
  if (max < 0) invalid("max < 0");
  if (max > 0 && (!tickets || !res)) invalid("tickets and res are required when max > 0");
  CGL_HIP(hipSetDevice(srv->ctx->device));
  admit_round(*srv);
  plain_round(*srv);
  run_round(*srv);
  // results are taken in completion order while their solution fits the caller's stride: the
  // first one that does not stays queued (and is refused here only when it is the first)
  if (betas && max > 0 && !srv->done.empty() &&
      betas_stride < (int64_t)srv->done.front().beta.size())
    invalid("betas_stride is smaller than the p of the next result");
  int32_t n = 0;
  while (n < max && !srv->done.empty()) {
    Finished& f = srv->done.front();
    if (betas && betas_stride < (int64_t)f.beta.size()) break;
    tickets[n] = f.ticket;
    res[n] = f.res;
    if (betas) std::copy(f.beta.begin(), f.beta.end(), betas + (int64_t)n * betas_stride);
    if (latency_s) latency_s[n] = f.latency;
    srv->done.pop_front();
    ++n;
  }
  *got = n;
  return CGL_OK;
  CGL_API_END
}

int cgl_server_cancel(cgl_server* srv, uint64_t ticket) {
  CGL_API_BEGIN
  if (!srv) invalid("NULL argument");
  for (auto it = srv->queue.begin(); it != srv->queue.end(); ++it) {
    if ((*it)->ticket != ticket) continue;
    std::unique_ptr<Request> r = std::move(*it);
    srv->queue.erase(it);
    cgl_result res{};
    res.lower_bound = -HUGE_VAL;
    res.primal = HUGE_VAL;
    res.gap_abs = HUGE_VAL;
    res.gap_rel = HUGE_VAL;
    res.status = CGL_CANCELLED;
    std::vector<double> beta((size_t)r->P->p, 0.0);
    finish(*srv, std::move(r), res, std::move(beta));
    return CGL_OK;
  }
  for (auto& R : srv->resident)
    for (auto& r : R.slot_req)
      if (r && r->ticket == ticket) {
        r->cancelled = true;  // retired with its best certified bound at the next round
        return CGL_OK;
      }
  set_error("unknown or finished ticket");
  return CGL_E_NOTFOUND;
  CGL_API_END
}

int cgl_server_stats(cgl_server* srv, int32_t* queued, int32_t* running, int32_t* done) {
  CGL_API_BEGIN
  if (!srv) invalid("NULL argument");
  int run = 0;
  for (const auto& R : srv->resident) run += R.running();
  if (queued) *queued = (int32_t)srv->queue.size();
  if (running) *running = run;
  if (done) *done = (int32_t)srv->done.size();
  return CGL_OK;
  CGL_API_END
}

int cgl_server_destroy(cgl_server* srv) {
  CGL_API_BEGIN
  if (!srv) return CGL_OK;
  (void)hipSetDevice(srv->ctx->device);
  for (auto& R : srv->resident) {
    // free the slots held by unfinished requests so the problem's engine stays usable
    MixedWork* W = R.P->mixed;
    if (!W) continue;
    for (int sl = 0; sl < W->S; ++sl)
      if (R.slot_req[(size_t)sl]) {
        W->st_host[sl].active = 0;
        W->slot_owner[(size_t)sl] = -1;
      }
    W->push_states(*R.P);
    CGL_HIP(hipStreamSynchronize(R.P->ctx->stream));
  }
  delete srv;
  return CGL_OK;
  CGL_API_END
}

}  // extern "C"

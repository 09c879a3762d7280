// Request server: continuous batching of node relaxations over resident problems.
//
// Submitted nodes wait in a FIFO queue. Every problem with queued or running mixed-precision
// nodes holds its batched engine (brought in while the device memory of the resident engines
// stays within the budget; an idle engine is released when another problem needs the room), and
// each resident engine runs on a HIP stream of its own, so engines of different designs advance
// independently and overlap on the device. An engine's turn, taken whenever its previous chunk
// has completed: take the chunk's outcome, run or queue its certification round, retire finished,
// certified or cancelled slots, admit queued nodes into free slots (at most max_slots per
// problem), and launch the next chunk of iterations. A poll starts the idle engines, solves one
// queued FP64-path node on the context's stream while the engines run, and then serves the
// engines whose chunks have completed (waiting for the first one if none has). Results wait in a
// completion list until polled. Calls on one server must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <memory>
#include <thread>
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

// A problem whose batched engine is resident, with the request held by each of its slots and
// the stream the engine runs on while the server holds it.
struct Resident {
  Problem* P = nullptr;
  hipStream_t stream = nullptr;
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

namespace cgl {
namespace {
// An FP64-path node in progress on a stream of its own (one per problem at a time: it uses the
// problem's plain-path buffers).
struct PlainJob {
  std::unique_ptr<Request> r;
  hipStream_t stream = nullptr;
};
}  // namespace
}  // namespace cgl

struct cgl_server {
  cgl_ctx* ctx = nullptr;
  size_t budget = 0;  // 0: no limit
  int max_slots = cgl::kSlots;
  uint64_t next_ticket = 1;
  std::deque<std::unique_ptr<cgl::Request>> queue;
  std::vector<cgl::Resident> resident;
  std::vector<cgl::PlainJob> plain_jobs;
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

// Hand the engine back to the context's stream and drop the server's stream (nothing of the
// engine is in flight).
void release_stream(Resident& R) {
  if (R.P->mixed) R.P->mixed->stream = R.P->ctx->stream;
  if (R.stream) {
    (void)hipStreamSynchronize(R.stream);
    (void)hipStreamDestroy(R.stream);
    R.stream = nullptr;
  }
}

// Queued mixed-precision nodes for P's engine (nodes of P or of a problem sharing its design).
bool has_queued(const cgl_server& S, const Problem* P) {
  for (const auto& r : S.queue)
    if (&r->P->engine_problem() == P && r->node.precision == CGL_PREC_MIXED) return true;
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
      if (R.running() == 0 && !has_queued(S, R.P) && !(R.P->mixed && R.P->mixed->in_flight)) {
        release_stream(R);
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
  CGL_HIP(hipStreamCreateWithFlags(&R.stream, hipStreamNonBlocking));  // default priority
  S.resident.push_back(std::move(R));
  return &S.resident.back();
}

// Engines for the problems of queued mixed-precision nodes, in queue order, as the budget allows.
void bring_in(cgl_server& S) {
  std::vector<Problem*> seen;
  for (const auto& q : S.queue) {
    if (q->node.precision != CGL_PREC_MIXED) continue;
    Problem* E = &q->P->engine_problem();
    if (std::find(seen.begin(), seen.end(), E) != seen.end()) continue;
    seen.push_back(E);
    make_resident(S, E);
  }
}

// Queued nodes of R's problem into its free slots (the engine is idle), in queue order.
void admit_for(cgl_server& S, Resident& R) {
  MixedWork& W = *R.P->mixed;
  std::vector<Admission> adm;
  for (auto it = S.queue.begin(); it != S.queue.end();) {
    Request& q = **it;
    const int member = W.member_of(q.P);
    if (member < 0 || q.node.precision != CGL_PREC_MIXED) {  // another engine's node
      ++it;
      continue;
    }
    if (R.running() >= S.max_slots) break;
    int slot = -1;
    for (int sl = 0; sl < W.S; ++sl)
      if (W.slot_owner[(size_t)sl] < 0 && !R.slot_req[(size_t)sl]) { slot = sl; break; }
    if (slot < 0) break;
    adm.push_back(Admission{slot, slot, q.node, q.host, member});
    R.slot_req[(size_t)slot] = std::move(*it);
    it = S.queue.erase(it);
  }
  W.admit(*R.P, adm);
}

// Finished, certified or cancelled slots of R to the completion list (the engine is idle).
void retire_for(cgl_server& S, Resident& R) {
  Problem& P = *R.P;
  MixedWork& W = *P.mixed;
  std::vector<int> done;
  for (int sl = 0; sl < W.S; ++sl) {
    const std::unique_ptr<Request>& r = R.slot_req[(size_t)sl];
    if (r && (W.st_host[sl].done || r->cancelled)) done.push_back(sl);
  }
  if (done.empty()) return;
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
  // a cancelled slot still runs on the device until its state says inactive
  W.push_states(P);
  CGL_HIP(hipStreamSynchronize(W.stream));
}

// One turn of an engine that has no work in flight (see the file comment).
void engine_turn(cgl_server& S, Resident& R) {
  Problem& P = *R.P;
  MixedWork& W = *P.mixed;
  W.stream = R.stream;
  if (W.in_flight) W.finish_chunk(P);
  W.set_relaxation(P);  // the shift changes only while the engine holds no node
  W.set_chunk(W.serve_chunk);
  if (W.cert_round(P, /*overlap=*/true) == MixedWork::kRoundOpen) {
    W.launch_chunk(P);  // queued behind the round; retirement after it
    return;
  }
  retire_for(S, R);
  admit_for(S, R);
  if (R.running() > 0) W.launch_chunk(P);
}

// Queued FP64-path nodes start, one per problem at a time, in queue order.
void plain_start(cgl_server& S) {
  for (auto it = S.queue.begin(); it != S.queue.end();) {
    Request& q = **it;
    if (q.node.precision == CGL_PREC_MIXED || q.P->plain.busy) {
      ++it;
      continue;
    }
    PlainJob job;
    job.r = std::move(*it);
    it = S.queue.erase(it);
    Problem& P = *job.r->P;
    CGL_HIP(hipStreamCreateWithFlags(&job.stream, hipStreamNonBlocking));  // default priority
    P.plain.busy = true;
    plain_begin(P, job.r->node, job.r->host, job.stream);
    plain_launch(P, job.stream);
    S.plain_jobs.push_back(std::move(job));
  }
}

// The plain jobs whose chunks have completed: finished (or cancelled) ones to the completion
// list, the others launch their next chunk.
void plain_serve(cgl_server& S, bool& any, bool& served) {
  for (size_t i = 0; i < S.plain_jobs.size();) {
    PlainJob& job = S.plain_jobs[i];
    Problem& P = *job.r->P;
    any = true;
    const hipError_t q = hipEventQuery(P.plain.chunk_ev);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    CGL_HIP(q);
    served = true;
    const bool finished = plain_after_chunk(P);
    if (!finished && !job.r->cancelled) {
      plain_launch(P, job.stream);
      ++i;
      continue;
    }
    cgl_result res{};
    std::vector<double> beta((size_t)P.p);
    plain_end(P, &res, beta.data(), job.stream);
    if (job.r->cancelled) res.status = CGL_CANCELLED;
    P.plain.busy = false;
    (void)hipStreamDestroy(job.stream);
    finish(S, std::move(job.r), res, std::move(beta));
    S.plain_jobs.erase(S.plain_jobs.begin() + (ptrdiff_t)i);
  }
}

void run_round(cgl_server& S) {
  // idle engines with work take a turn (their chunks then run while the host goes on), and
  // queued FP64-path nodes start on streams of their own
  for (auto& R : S.resident)
    if (!R.P->mixed->in_flight && (R.running() > 0 || has_queued(S, R.P))) engine_turn(S, R);
  plain_start(S);
  // engines and plain jobs whose chunks have completed are served; wait for the first one if
  // none has
  for (;;) {
    bool any = false, served = false;
    plain_serve(S, any, served);
    for (auto& R : S.resident) {
      MixedWork& W = *R.P->mixed;
      if (!W.in_flight) continue;
      any = true;
      const hipError_t q = hipEventQuery(W.chunk_done);
      if (q == hipErrorNotReady) continue;
      CGL_HIP(q);
      engine_turn(S, R);
      served = true;
    }
    if (!any || served) return;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
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
  bring_in(*srv);
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
  for (auto& job : srv->plain_jobs)
    if (job.r->ticket == ticket) {
      job.r->cancelled = true;  // stopped after its chunk in flight, with its best bound
      return CGL_OK;
    }
  set_error("unknown or finished ticket");
  return CGL_E_NOTFOUND;
  CGL_API_END
}

int cgl_server_stats(cgl_server* srv, int32_t* queued, int32_t* running, int32_t* done) {
  CGL_API_BEGIN
  if (!srv) invalid("NULL argument");
  int run = (int)srv->plain_jobs.size();
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
  for (auto& job : srv->plain_jobs) {
    CGL_HIP(hipStreamSynchronize(job.stream));
    job.r->P->plain.busy = false;
    (void)hipStreamDestroy(job.stream);
  }
  srv->plain_jobs.clear();
  for (auto& R : srv->resident) {
    // free the slots held by unfinished requests so the problem's engine stays usable
    MixedWork* W = R.P->mixed;
    if (!W) continue;
    W->stream = R.stream;
    if (W->in_flight) {
      CGL_HIP(hipEventSynchronize(W->chunk_done));
      W->finish_chunk(*R.P);
    }
    for (int sl = 0; sl < W->S; ++sl)
      if (R.slot_req[(size_t)sl]) {
        W->st_host[sl].active = 0;
        W->slot_owner[(size_t)sl] = -1;
      }
    W->push_states(*R.P);
    CGL_HIP(hipStreamSynchronize(R.stream));
    release_stream(R);
  }
  delete srv;
  return CGL_OK;
  CGL_API_END
}

}  // extern "C"

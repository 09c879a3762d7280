// Host side of the batched mixed-precision engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "engine.h"
#include "mixed.h"

namespace cgl {

constexpr int kSlots = 256;  // node slots per problem
constexpr int kChunk = 4;       // iterations per graph launch between host checks: the server
constexpr int kSolveChunk = 8;  // ... a batched solve (cgl_solve_batch), where throughput counts
constexpr int kCertBatch = 16;  // certification requests that trigger a round at once
constexpr int kCertWait = 1;    // chunks the oldest request may wait for others
constexpr int kReorderEvery = 8;  // cycles between checks of the X-pass operand order
// a reorder is made when the union is at least 1 / kReorderShrink of the extent shorter
constexpr int kReorderShrink = 8;
constexpr int64_t kGramMaxP = 20480;  // least squares: largest p with an FP64 Gram matrix (3.4 GB)

struct Admission {
  int slot;
  int owner;  // caller's index (solve) or request id (server)
  cgl_node node;
  NodeHost host;
  int member = 0;  // index of the node's problem among the engine's problems
};

// Device buffers of one problem served by an engine (labels and cold-start base).
struct MemberBufs {
  DevBuf y, H0c, b0c, b1c;
};

struct MixedWork {
  bool ready = false;
  int S = 0, S_pad = 0;
  int64_t n_pad = 0, ldp = 0;
  int ksplit = 1;
  int64_t xt_kchunk = 0;
  int nrt = 0, ncchunk = 0, ksx = 1;
  int64_t x_kchunk = 0;
  int64_t rchunk = 0, cchunk = 0;
  // the problems served (members[0] is the engine's own; the others share its design), their
  // buffers and the device table the kernels read (a slot's state names its problem)
  std::vector<Problem*> members;
  std::vector<std::unique_ptr<MemberBufs>> mbufs;
  MemberDev mem_host[kMaxMembers] = {};
  DevBuf memtab;
  int member_of(const Problem* Q) const;  // index in members, -1 if not served
  void forget_member(const Problem* Q);    // a sharer is destroyed: no more nodes of it come
  DevBuf Xb, Xbt, st, cls, bring, beta0, H0, base0, base1, e0f, bres, bdual, dop, gop, gop_r, gsel, dU, dUp, dH, lpart, npart,
      fpart, cycle, prevsel, B64, U64, R64, H64, cpart, list, Xt, part64,
      sflag, sidx, scount, Bu, G, Bret, pinv, pinv_new, perm, perm_new, dop_tmp, pfx, sj, sv;
  int64_t ldg = 0;  // least squares: G = X^T X in FP64 (p x ldg), when built
  size_t part64_cap = 0;
  NodeDev* st_host = nullptr;
  double* beta_host = nullptr;  // pinned staging of retired iterates (S x p)
  int* count_host = nullptr;    // pinned: size of the support union of a certification round
  hipStream_t copy_stream = nullptr;  // deferred copies of retired iterates (default priority)
  hipEvent_t ret_gathered = nullptr, ret_copied = nullptr;
  bool ret_copy_recorded = false;
  std::vector<double*> ret_pending;  // callers' buffers of the staged rows, in row order
  int64_t pending_p = 0;
  int64_t support_sum = 0;      // sum over certification rounds of the union size (statistics)
  int* order_host = nullptr;    // pinned: staging of the support prefix
  int ext_seen[2] = {0, 0};     // X-pass extent statistics already accounted
  // st holds the S slot states and then a control tail of ints that every state copy to the host
  // brings along: the X-pass extent counters and statistics, the union size of the last reorder
  // check and the strays per slot (copies to the device write the states only)
  static constexpr int kCtlExtent = 0, kCtlUnion = 4, kCtlStrays = 8;
  size_t st_bytes() const { return (size_t)S * sizeof(NodeDev) + (size_t)(kCtlStrays + S) * sizeof(int); }
  int* ctl_dev() const { return (int*)((char*)st.ptr + (size_t)S * sizeof(NodeDev)); }
  const int* ctl_host() const { return (const int*)((const char*)st_host + (size_t)S * sizeof(NodeDev)); }
  bool reorder = true;          // CGL_NO_REORDER=1 keeps the natural coordinate order
  int64_t reorder_checked = 0;  // cycle of the last reorder check
  int64_t reorders = 0;
  int64_t prefix_cap = 0;       // CGL_PREFIX_CAP (tests): upper bound of the support prefix
  uint8_t* cls_host = nullptr;  // pinned: S x ldp node classes (rows uploaded at admission)
  // pinned staging of slot lists, one region of S per caller (certification, retirement,
  // admission); a region is reused only after a synchronisation that follows its copy
  int* list_host = nullptr;
  enum { kListCert = 0, kListRetire = 1, kListAdmit = 2 };
  void upload_list(Problem& P, const std::vector<int>& v, int region);
  std::vector<int> slot_owner;
  int64_t admitted_at[kSlots] = {0};
  int64_t want_since[kSlots];  // cycle at which a slot's certification request was first seen
  int64_t cycles = 0;
  int64_t cert_rounds = 0;
  int cert_batch = kCertBatch;  // CGL_CERT_BATCH overrides
  int cert_wait = kCertWait;    // CGL_CERT_WAIT overrides
  int chunk = kChunk;           // cycles per launch between host checks (the one in use)
  int serve_chunk = kChunk;     // the server's and a batched solve's; CGL_CHUNK overrides both
  int solve_chunk = kSolveChunk;
  void set_chunk(int c);        // a captured chunk of another length is dropped
  int reorder_every = kReorderEvery;  // CGL_REORDER_EVERY overrides
  int reorder_shrink = kReorderShrink;  // CGL_REORDER_SHRINK overrides
  hipGraphExec_t graph_exec = nullptr;  // one chunk of cycles
  MixedDev md{};

  // Tilings of the two products, as codes: the split-K, plus kTile128 for the 128-row tile and
  // 2 kTile128 for the 64-row tile (else 256 rows). The autotuner picks one code per product
  // shape.
  static constexpr int kTile128 = 100;
  static int code_rt(int code) { return 8 >> std::min(code / kTile128, 2); }
  static int code_ks(int code) { return code % kTile128; }
  std::vector<int> split_cands_x, split_cands_xt;
  static std::vector<int> split_candidates(int64_t m_tiles, int64_t K);
  static std::vector<int> tiling_candidates(int64_t M, int64_t K);
  void set_split_x(int code);
  void set_split_xt(int code);
  void tune_splits(Problem& P);
  void ensure(Problem& P);
  // Take the problem's step size and eigen-perspective shift (they change with
  // cgl_problem_set_eigen); a captured chunk is re-captured. Only while nothing is in flight.
  void set_relaxation(Problem& P);
  // All of the engine's device work goes to `stream`: the context's stream, or a stream of its
  // own while a server holds the engine (set only while no work of the engine is in flight).
  hipStream_t stream = nullptr;
  // One chunk of cycles: launch_chunk queues it (with the reorder probe and the copy of the slot
  // states to the host) and records chunk_done; finish_chunk, once that event has completed,
  // takes the chunk's outcome (the open certification round, the operand order, statistics).
  // run_chunk does both and waits in between.
  hipEvent_t chunk_done = nullptr;
  bool in_flight = false;
  bool chunk_probe = false;
  void launch_chunk(Problem& P);
  void finish_chunk(Problem& P);
  void run_chunk(Problem& P);
  // Certification round for the nodes that asked (see the batching rule in the source). With
  // overlap, a round that leaves other nodes running is only queued (kRoundOpen): the next
  // run_chunk's synchronisation brings its outcome and closes it.
  enum { kRoundNone = 0, kRoundDone = 1, kRoundOpen = 2 };
  int cert_round(Problem& P, bool overlap = false);
  void close_round(Problem& P);
  bool round_open = false;
  bool round_span = false;  // the open round's GPU span is being timed (profiling level 3)
  // X-pass operand order. The probe (queued at the end of a chunk) lists the coordinates where a
  // running slot's recent iterates, base point or operand are nonzero and stages the extent and
  // stray counts for the host; after the chunk's synchronisation, apply puts those coordinates
  // first (the columns of Xb alike, the support prefix at their count) when that shortens the
  // operand's extent by an eighth or the strays have piled up.
  void reorder_probe(Problem& P);
  void reorder_apply(Problem& P);
  void admit(Problem& P, const std::vector<Admission>& adm);
  // Results of finished slots and their best certified iterates (beta_out[i] may be null): one
  // gather of the iterates on the device, one copy to pinned host memory, then into the
  // callers' buffers. The slots are freed. With defer, the copy runs on a stream of its own while
  // the next launches proceed, and the iterates reach the callers' buffers at flush_retired()
  // (called before the next retirement and before the solve returns).
  // dual_out (optional, entries may be null): the iterate whose dual point gave each slot's
  // certified bound, copied synchronously.
  void retire(Problem& P, const std::vector<int>& slots, const std::vector<cgl_result*>& res,
              const std::vector<double*>& beta_out, bool defer = false,
              const std::vector<double*>* dual_out = nullptr);
  void flush_retired();
  void drop_retired();  // forget staged iterates (their copy is waited for first)
  void push_states(Problem& P);
  int free_slots() const;
  size_t device_bytes() const;  // device memory held by this engine
  ~MixedWork();
};

}  // namespace cgl

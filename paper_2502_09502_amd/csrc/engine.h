// Host-side engine objects of libcertglm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <array>
#include <map>
#include <vector>

#include "../../include/certglm.h"
#include "kernels.h"
#include "solver.h"

struct cgl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // kernel timing (cgl_ctx_set_profiling)
  bool profiling = false;    // levels 1 and 2: kernel events (launches outside graphs)
  bool profile_x = false;    // level 2: the batched X pass is timed too
  bool phase_timing = false; // levels 1 to 3: host wall time of the batched engine's phases
  double kt_ms[16] = {0};
  int64_t kt_n[16] = {0};
  std::vector<hipEvent_t> events;  // pool, grown on demand
  hipEvent_t event(size_t i);
  // split-K choices of the batched products found by timing, by (pass, M, K, nodes); loaded
  // from and appended to the tuning cache file (tune_cache_path) for this device's architecture
  std::map<std::array<int64_t, 4>, int> tuned_split;
  int tiling[2] = {0, 0};  // tiling codes of the last batched engine set up (X pass, X^T pass)
  std::string arch;  // gcnArchName up to the first ':' (e.g. "gfx950")
  void load_tuning();
  void save_tuning(const std::array<int64_t, 4>& key, int choice) const;
  ~cgl_ctx();
};

namespace cgl {

struct InvalidArg {
  std::string msg;
};
[[noreturn]] void invalid(const std::string& m);

// Owning device allocation.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  void alloc(size_t b);
  void reset();
  template <typename T>
  T* as() const { return static_cast<T*>(ptr); }
};

int64_t pad_cols(int64_t p);

// Validated node on the host.
struct NodeHost {
  std::vector<uint8_t> cls;  // per coordinate: CLS_FREE / CLS_ZERO / CLS_ONE
  int kp = 0;                // k - |Z1|
  int nfree = 0;
  bool infeasible = false;
};

NodeHost make_node_host(const cgl_node& nd, int64_t p, int k);
NodeDev make_node_dev(const cgl_node& nd, const NodeHost& h);
void fill_result(const NodeDev& s, cgl_result* r);
// Takes this device's address of the allocation-free prox's scratch array (noalloc.hip); called
// once per context creation with the device current.
void noalloc_setup(int device);
void infeasible_result(cgl_result* r, double* beta_out, int64_t p);

struct Problem;

// Workspace of the plain per-node path (reused across solves of one problem).
struct PlainWork {
  static constexpr int kChunk = 8;  // iterations per launch between host checks
  bool ready = false;
  bool busy = false;  // a server's plain solve of this problem is in progress
  PlainGeom geom{};
  DevBuf bring, uring, bbest, w, h, part, fpart, lpart, cls, st, gsq;
  NodeDev* st_host = nullptr;
  NodeDev st0{};              // staging of the initial state (read by an asynchronous copy)
  std::vector<double> warm;   // staging of a warm start
  hipGraphExec_t graph_exec = nullptr;
  hipEvent_t chunk_ev = nullptr;
  int iter_before = 1;
  void ensure(Problem& P);
  ~PlainWork();
};

struct MixedWork;  // batch.cpp

struct Problem {
  cgl_ctx* ctx = nullptr;
  int64_t n = 0, p = 0, ldx = 0;
  int xtype = XT_F64;
  int loss = LOSS_LS;
  double lam2 = 0, M = 0, L = 0, rho = 0;
  int k = 0;
  DevBuf X;  // n x ldx in the stored precision, zero padded
  DevBuf y;  // n doubles
  PlainWork plain;
  double shift = 0.0;          // eigen-perspective shift s (App. D.2); 0: perspective relaxation
  double lam_max = 0.0;        // lambda_max(X^T X) estimate when the library computed L
  MixedWork* mixed = nullptr;  // created on first mixed solve
  size_t mixed_bytes = 0;      // its device footprint, once known
  // Problems on the same design (cgl_problem_share_design): an owner's batched engine serves
  // its sharers' mixed-precision nodes too; a sharer names its owner and has no engine.
  std::vector<Problem*> sharers;
  Problem* design_owner = nullptr;
  Problem& engine_problem() { return design_owner ? *design_owner : *this; }
  ~Problem();
};

void solve_plain(Problem& P, const cgl_node& nd, const NodeHost& nh, double* beta_out,
                 cgl_result* res);
// solve_plain in steps on a stream (see api.cpp): begin, then launch / (chunk_ev completes) /
// after_chunk until it returns true, then end.
void plain_begin(Problem& P, const cgl_node& nd, const NodeHost& nh, hipStream_t s);
void plain_launch(Problem& P, hipStream_t s);
bool plain_after_chunk(Problem& P);
void plain_end(Problem& P, cgl_result* res, double* beta_out, hipStream_t s);
// Batched solve of count mixed-precision nodes; node i's result and solution go to row rows[i]
// of res and beta_out (row i when rows is null), and with dual_out the iterate whose dual point
// gave its certified bound to the same row of dual_out.
void solve_mixed(Problem& P, const cgl_node* nodes, int32_t count, double* beta_out,
                 cgl_result* res, const int32_t* rows = nullptr, double* dual_out = nullptr);
void certify_host_beta(Problem& P, const NodeHost& nh, const double* beta, double* primal,
                       double* dual);
// G = X^T X in FP64 (p rows, leading dimension ldg), from the transposed design xt (p x n_pad,
// the stored precision, zero past column n): rows of 256 widened, then the FP64 MFMA product
// (part: split-K scratch of cap bytes). Synchronises the stream before it returns.
void build_gram(int xtype, const void* xt, int64_t n_pad, int64_t n, int64_t p, double* G,
                int64_t ldg, double* part, size_t cap, hipStream_t s);
// Eigen-perspective shift (App. D.2): whether s <= lambda_min(X^T X) is proved by an FP64
// Cholesky factorisation (eigen.cpp), and the largest shift such a factorisation proves.
bool eigen_shift_proved(Problem& P, double shift);
double eigen_shift_certified(Problem& P, double rel_tol);

}  // namespace cgl

// Every extern "C" entry point body sits between these: C++ exceptions become status codes
// (with the detail string for cgl_last_error) and never cross the ABI.
#define CGL_API_BEGIN try {
#define CGL_API_END                                                       \
  }                                                                       \
  catch (const ::cgl::InvalidArg& e) {                                           \
    ::cgl::set_error(e.msg);                                                     \
    return CGL_E_INVAL;                                                   \
  }                                                                       \
  catch (const ::cgl::HipError& e) {                                             \
    ::cgl::set_error(std::string(e.what) + ": " + hipGetErrorString(e.err));     \
    return e.err == hipErrorOutOfMemory ? CGL_E_NOMEM : CGL_E_DEVICE;     \
  }                                                                       \
  catch (const std::bad_alloc&) {                                         \
    ::cgl::set_error("allocation failed");                                       \
    return CGL_E_NOMEM;                                                   \
  }                                                                       \
  catch (const std::exception& e) {                                       \
    ::cgl::set_error(e.what());                                                  \
    return CGL_E_INTERNAL;                                                \
  }                                                                       \
  catch (...) {                                                           \
    ::cgl::set_error("unknown error");                                           \
    return CGL_E_INTERNAL;                                                \
  }

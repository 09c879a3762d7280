// Device view of the batched mixed-precision engine and its launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "solver.h"

namespace cgl {

constexpr int kStallCycles = 6;   // re-centre when the working gap has not halved for this long
constexpr double kCertGap = 1.0;  // ask for an FP64 round once the working gap is <= kCertGap * tol
constexpr double kRestartSlack = 1.5;  // noise margin of the restart test (0: plain comparison)

// One problem served by an engine: the problems of an engine share the design X and differ in
// the labels, the loss and the constants. A slot's state names its problem (NodeDev::member).
constexpr int kMaxMembers = 4;
struct MemberDev {
  const double* y;    // n_pad labels (zero padded)
  const double* H0c;  // ldp: X^T grad f(0), the base gradient of a cold start
  const double* b0c;  // n_pad: least squares e_0 = -y; other losses u_0 = 0
  const double* b1c;  // n_pad: other losses r_0 = grad f(0)
  int loss;
  double lam2, M, L, rho;
  double shift;       // eigen-perspective shift s (App. D.2; least squares), 0 otherwise: the
                      // gradient gains -2 s gamma, the objective -s ||beta||^2, the regulariser
                      // weight is 2 (lambda2 + s) and the bound gains s ||point||^2
};

struct MixedDev {
  // problem
  const uint16_t* Xb;   // n_pad x ldp, BF16 copy of X (zero padded)
  const uint16_t* Xbt;  // ldp x n_pad, its transpose
  int64_t n, p, n_pad, ldp;
  const MemberDev* mem; // kMaxMembers entries (device)
  int loss_kinds;       // bit 0: a problem with least squares; bit 1: one with another loss
  double cert_gap;      // a node asks for an FP64 round when its working gap is <= cert_gap * tol
  int stall_cycles;     // ... or when that gap has not halved for this many cycles
  // slots
  int slots;            // S
  int S_pad;            // operand rows, multiple of 256
  NodeDev* st;          // S
  const uint8_t* cls;   // S x ldp
  double* bring;        // 3 rings x S x ldp (FP64 iterates)
  int64_t bring_stride; // S x ldp
  double* beta0;        // S x ldp base point
  double* H0;           // S x ldp: X^T grad f(X beta_0)
  double* base0;        // S x n_pad: u_0 = X beta_0 (losses other than least squares)
  float* e0f;           // S x n_pad: least squares e_0 = X beta_0 - y, rounded to FP32 (its
                        // rounding is the same in every cycle between re-centres)
  double* base1;        // S x n_pad: logistic r_0 = grad f(u_0)
  double* bres;         // S x ldp: best certified iterate
  double* bdual;        // S x ldp: the iterate whose dual point zeta = -grad f(X beta) gave the
                        // best certified bound
  uint16_t* dop;        // S_pad x ldp: bf16(beta - beta_0)
  uint16_t* gop;        // S_pad x n_pad: bf16(grad f(u_gamma) - r_0) without a restart
  uint16_t* gop_r;      // S_pad x n_pad, slot-major: the same after a restart (c = 1/4)
  int* gsel;            // S_pad: 1 where this cycle's restart test restarted (gop_r was copied
                        // into gop; the node kernel reads F* partial set 1)
  float* dU;            // 2 rings x S_pad x n_pad
  int64_t dU_ring;
  float* dUp;           // ksx x S_pad x n_pad split-K partials of the X pass
  int64_t dUp_split;
  int ksx;
  int64_t x_kchunk;
  int x_rt;             // row tiles of 32 per wave of the X pass's product (8 or 4)
  float* dH;            // ksplit x S_pad x ldp split-K partials of the X^T pass
  int64_t dH_split;
  int ksplit;
  int64_t xt_kchunk;
  int xt_rt;            // the same for the X^T pass
  double* lpart;        // S x nrt loss partials
  double* npart;        // S x nrt: sums of (f_i'(u) dU_i)^2, the scale of the loss's rounding
  double restart_slack; // > 0: a restart needs L^{t+1} >= L^t + slack 2^-9 sqrt(sum npart)
  double* fpart;        // S x 2 x nrt F* partials at gamma (loss kernel; set 1: after a restart)
  int nrt;
  int64_t rchunk;
  int* cycle;           // cycle counter: the cycle running, or between cycles the last one run
  int* prevhead;        // S x 65: last prox head selection (count, indices) per slot
  int* prevtop;         // S x 65: last top-k' selection of the dual monitor per slot
  // X-pass operand order: coordinate j sits at operand position pinv[j] (the columns of Xb are
  // permuted alike; identity past p), and the operand is zero at positions >= max(keff[0],
  // keff[1]). The node kernel of cycle t raises keff[(t + 1) & 1]; the loss kernel of cycle t
  // clears keff[t & 1] after the X pass of cycle t has read it.
  const int* pinv;      // ldp
  const int* perm;      // ldp: the coordinate at each operand position
  int* keff;            // 2 counters, then the extent statistics (columns / 128, passes)
  // Operand entries at positions >= *pfx (the support prefix of the current order) leave the
  // operand as strays: up to kStrayCap per slot, as (coordinate, value) pairs that the loss
  // kernel adds to the X-pass product (X~ column from the rows of X~^T); a slot with more keeps
  // the rest in the operand, which the extent then covers.
  const int* pfx;       // 1
  int* sn;              // S: strays of the operand in flight
  int* sj;              // S x kStrayCap coordinates
  float* sv;            // S x kStrayCap values (BF16-rounded)
};

constexpr int kStrayCap = 64;
constexpr int kLossChunk = 1024;  // rows per block of the loss kernel (4 per thread)

void launch_make_bf16(int xtype, const void* X, int64_t ldx, int64_t n, int64_t p, int64_t n_pad,
                      int64_t ldp, uint16_t* Xb, uint16_t* Xbt, hipStream_t s);
// advance: the launch also advances the cycle counter (the first launch of a cycle). e0, e1
// (optional): events that the launch itself updates with the kernel's start and end.
void launch_gemm_x(const MixedDev& md, hipStream_t s, bool advance = false,
                   hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_gemm_xt(const MixedDev& md, hipStream_t s, hipEvent_t e0 = nullptr,
                    hipEvent_t e1 = nullptr);
void launch_mixed_loss(const MixedDev& md, hipStream_t s);
void launch_mixed_decide(const MixedDev& md, hipStream_t s);
void launch_mixed_node(const MixedDev& md, hipStream_t s);
// C[q][m] = sum_k A[m][k] B[q][k] in FP64 (A row-major in the design's stored precision);
// part: split-K scratch of part_cap bytes (the split is limited to what fits).
void launch_gemm_f64(int xtype, const void* A, int64_t lda, int64_t M, int64_t K,
                     const double* B, int64_t ldb, int Q, double* C, int64_t ldc, double* part,
                     size_t part_cap, hipStream_t s);
// C[q][m] = sum_{u < K} At[idx[u]][m] B[q][u] in FP64: the product with right-hand sides that
// are zero outside the coordinates idx (At: transposed design, ldat >= M rounded up to 256;
// idx readable up to K rounded up to 16; B compacted to those coordinates). With kdev, K is read
// from device memory at launch (at most the K given, which sets the launch shape).
void launch_gemm_f64_rows(int xtype, const void* At, int64_t ldat, const int* idx, int64_t M,
                          int64_t K, const int* kdev, const double* B, int64_t ldb, int Q,
                          double* C, int64_t ldc, double* part, size_t part_cap, hipStream_t s);
// dst[r][c] = src[r][c] (the design's stored precision) widened to FP64, r < rows, c < cols.
void launch_widen(int xtype, const void* src, int64_t ld, int64_t rows, int64_t cols, double* dst,
                  int64_t ldd, hipStream_t s);
// Least squares: H[q][j] = 2 H[q][j] + h0[j] for j < p (H = X^T X beta on entry, h0 = -2 X^T y of
// the problem of slot list[q]).
void launch_gram_finish(double* H, int64_t ld, int64_t p, int nq, const MixedDev& md, const int* list,
                        hipStream_t s);
// Xt (p x n_pad) = X^T in the stored precision, zero in columns n .. n_pad.
void launch_transpose(int xtype, const void* X, int64_t ldx, int64_t n, int64_t p, int64_t n_pad,
                      void* Xt, hipStream_t s);
// B64 rows = the latest iterates of the listed slots; flag[j] = 1 where one of them is nonzero.
void launch_cert_gather(const MixedDev& md, const int* list, int nq, double* B64, uint8_t* flag,
                        hipStream_t s);
// idx = the flagged coordinates in order (zero padded to a multiple of 16), *count = their
// number; clears the flags.
void launch_cert_support(uint8_t* flag, int64_t p, int* idx, int* count, hipStream_t s);
// Bu[q][u] = B64[q][idx[u]] for u < K = *kdev (K <= Kmax), zero up to K rounded up to 16
// (leading dimension ld).
void launch_cert_compact(const double* B64, int64_t ld, const int* idx, const int* kdev,
                         int64_t Kmax, int nq, double* Bu, hipStream_t s);
void launch_cert_resid(const MixedDev& md, const int* list, int nq, const double* U64,
                       double* R64, double* part, int nchunk, int64_t chunk, hipStream_t s);
void launch_cert_finish(const MixedDev& md, const int* list, int nq, const double* B64,
                        const double* H64, const double* part, int nchunk, hipStream_t s);
void launch_slot_clear(const MixedDev& md, int slot, hipStream_t s);
// Operand order by support: flag[j] = 1 where one of a running slot's last three iterates, its
// base point or its operand in flight (strays included) is nonzero; then perm (position -> coordinate) and pinv (coordinate -> position) with the flagged
// coordinates first, each group in increasing order (identity past p), *count = their number;
// the flags are cleared.
void launch_perm_flags(const MixedDev& md, uint8_t* flag, hipStream_t s);
void launch_perm_build(uint8_t* flag, int64_t p, int64_t ldp, int* perm, int* pinv, int* count,
                       hipStream_t s);
// Re-lay the operand of every slot from the order pinv_old (a copy in dop_old) to pinv_new and
// raise both extent counters to one past the last nonzero position.
void launch_perm_operand(const MixedDev& md, const uint16_t* dop_old, const int* pinv_old,
                         const int* pinv_new, hipStream_t s);
// Xb[i][u] = Xbt[perm[u]][i] for u < p (columns past p keep their zeros).
void launch_perm_design(const uint16_t* Xbt, int64_t n_pad, const int* perm, int64_t p,
                        uint16_t* Xb, int64_t ldp, hipStream_t s);
// dst (nq x p, contiguous) = rows list[q] of src (leading dimension ld).
void launch_gather_rows(const double* src, int64_t ld, const int* list, int nq, int64_t p,
                        double* dst, hipStream_t s);
void launch_admit(const MixedDev& md, const int* list, int nq, hipStream_t s);

}  // namespace cgl

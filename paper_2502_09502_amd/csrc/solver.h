// Device-side state and kernel launchers shared by the plain (FP64 per node) and the batched
// mixed-precision paths.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cgl {

enum LossKind : int { LOSS_LS = 0, LOSS_LOGISTIC = 1, LOSS_SQHINGE = 2, LOSS_POISSON = 3, LOSS_GAMMA = 4 };
enum XType : int { XT_F64 = 0, XT_F32 = 1, XT_BF16 = 2 };

// Per-node iteration state of Alg. 3, resident in device memory.
struct NodeDev {
  double phi;        // momentum counter (Alg. 3): c = phi / (phi + 3)
  double c;          // momentum coefficient used by the current iteration
  double L_prev;     // objective at beta^t
  double g_new;      // g_node(beta^{t+1}) from the prox
  double gstar_new;  // g_node*(v / (2 lambda2)) of the dual monitor, when checked
  double fstar_new;  // F*(-zeta) of the dual monitor
  double P_best;     // best primal value so far
  double D_best;     // best dual value so far
  double L_work;     // last working-precision objective
  double vstar;      // pooled prox value of the last iteration (warm start of the next)
  int iter;          // t (1-based): beta^t is the current iterate
  int restarts;
  int status;        // cgl_node_status; -1 while running
  int done;
  int checked;       // the dual monitor ran in the current iteration
  int best_iter;
  int kp;            // k - |Z1|
  int nfree;         // |F|
  int max_iter;
  int check_every;
  int recentres;
  int want_cert;     // mixed path: the node asks for an FP64 re-centring / certificate
  double tol;
  double incumbent;
  // mixed path
  double P_cert;     // best FP64-certified primal value
  double D_cert;     // best FP64-certified dual value
  double mgap_ref;   // working gap at the last halving
  int active;        // slot holds a node whose base point is set
  int primed;        // L^t of the current base is known (no restart test before that)
  int since_improve; // cycles since the working gap last halved
  int since_recentre;
  int b_int0;        // scratch flag of the certification kernel
  int last_ring;     // ring slot holding the latest prox output (the iterate g_new belongs to)
  int need_base;     // warm start admitted: parked until an FP64 round sets its base point
  double bsq_new;    // ||beta^{t+1}||^2 (eigen-perspective objective)
  int rebase;        // mixed path: the base moved under a running momentum (next cycle only)
  // mixed path: restart-test outcome of the current cycle, taken by the decision kernel from the
  // state above and committed by the node kernel (phi, L^{t+1}, primed, restarts)
  double rs_phi;
  double rs_L;
  int rs_primed;
  int rs_restarts;
  int member;        // mixed path: the problem of the engine's member table the node belongs to
};

constexpr int kRunning = -1;

// Problem constants handed to kernels by value.
struct ProbParams {
  int64_t n, p, ldx, ldxt;  // padded leading dimensions
  double lam2, M, L, rho;
  int k;
  int loss;
  int xtype;
};

}  // namespace cgl

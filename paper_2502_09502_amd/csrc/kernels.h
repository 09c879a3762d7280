// Host-side launchers of the HIP kernels (implemented in kernels_*.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "solver.h"

namespace cgl {

struct PlainGeom {
  int64_t ntiles;      // column tiles of k_xt
  int nchunks;         // row chunks of k_xt (partials per column)
  int64_t chunk_rows;  // rows per chunk
  int nxb;             // workgroups of k_xb (loss partials)
};

int64_t xt_vec(int xtype);
PlainGeom plain_geometry(int xtype, int64_t n, int64_t p_pad);
int prox_elems(int64_t p);

void launch_xb(int xtype, const void* X, int64_t ldx, int64_t n, int64_t p_pad, const double* b,
               int64_t bs, double* u, int64_t us, const NodeDev* st, const double* y, int loss,
               double* loss_part, hipStream_t stream);
void launch_xt(int xtype, const void* X, int64_t ldx, int64_t n, int64_t p_pad,
               const PlainGeom& g, const double* u, int64_t us, const NodeDev* st,
               const double* y, int loss, int mode, double* part, double* fpart,
               hipStream_t stream);
void launch_grad_step(const double* part, int nchunks, int64_t p_pad, const NodeDev* st,
                      const double* b_base, int64_t b_stride, double inv_L, double* h, double* w,
                      hipStream_t stream, double shift = 0.0, double* gsq_part = nullptr);
void launch_prox(int nodes, const double* w, int64_t w_ld, const double* h, int64_t h_ld,
                 const uint8_t* cls, int64_t cls_ld, int64_t p, double rho, double M,
                 double two_l2, NodeDev* st, double* b_base, int64_t b_stride,
                 int64_t b_node_stride, hipStream_t stream, int want_bsq = 0);
// The node prox for p beyond one workgroup's per-thread values (prox_paged.hip): w, cls and b
// rows of the nodes at strides w_ld, cls_ld, b_ld; the states give k' and |F| and receive g and
// v*.
void launch_prox_paged(int nodes, const double* w, int64_t w_ld, const uint8_t* cls,
                       int64_t cls_ld, int64_t p, double rho, double M, NodeDev* st, double* b,
                       int64_t b_ld, hipStream_t stream);
// In-place FP64 Cholesky factorisation of A - shift I (p x p, lower triangle, leading dimension
// lda) on the stream; *fail (zero on entry) becomes 1 at the first non-positive pivot
// (chol.hip).
void launch_chol_factor(double* A, int64_t lda, int64_t p, double shift, int* fail,
                        hipStream_t s);
void launch_finish(const double* loss_part, int nloss, const double* fstar_part, int nfstar,
                   double two_l2, NodeDev* st, const double* b_base, int64_t b_stride,
                   double* b_best, int64_t p, hipStream_t stream, double shift = 0.0,
                   const double* gsq_part = nullptr, int ngsq = 0);
void launch_init_state(const double* loss_part, int nloss, double L0_g, NodeDev* st,
                       hipStream_t stream);

void launch_power_normalize(const double* z, double* v, int64_t p, double* lam,
                            hipStream_t stream);
void launch_resid(const double* u, const double* y, int64_t n, int loss, double* r,
                  double* part2, hipStream_t stream);
void launch_g_gstar(int nodes, const double* beta, int64_t b_ld, const double* h, int64_t h_ld,
                    const uint8_t* cls, int64_t cls_ld, const NodeDev* st, int64_t p, double M,
                    double two_l2, double* out, hipStream_t stream);
// *bad += number of non-finite values among the count stored elements of X (BF16: exponent all
// ones); *bad must start at zero.
void launch_count_nonfinite(int xtype, const void* X, int64_t count, int* bad, hipStream_t s);
// diff += number of 32-bit words where two device buffers differ (words 32-bit words each).
void launch_count_diff(const void* a, const void* b, int64_t words, int* diff, hipStream_t s);

}  // namespace cgl

// Certified shift of the eigen-perspective relaxation (App. D.2): its bound needs
// Q = X^T X - s I positive semidefinite, i.e. s <= lambda_min(X^T X). A shift is accepted only
// when an FP64 Cholesky factorisation of G - (s + delta) I runs to completion on the device, with
// G = X^T X computed in FP64 from the stored values of X.
//
// Why that proves it. If Cholesky of B runs to completion in floating point, the computed factor
// satisfies L L^T = B + E with |E| <= gamma_{p+1} |L| |L|^T (the backward error bound of the
// Cholesky factorisation, Higham, Accuracy and Stability of Numerical Algorithms, Thm. 10.3; it
// holds for any order of the inner-product sums), and by Cauchy-Schwarz
// ||E||_2 <= gamma_{p+1} / (1 - gamma_{p+1}) trace(B). The FP64 product G differs from X^T X by
// at most gamma_n |X|^T |X| entrywise, whose 2-norm is at most gamma_n trace(X^T X). So
// lambda_min(X^T X) >= s + delta - (gamma_{p+1} / (1 - gamma_{p+1}) + gamma_n) trace(G) (1 + u),
// with gamma_k = k u / (1 - k u), u = 2^-53; delta = 4 (n + p + 2) u trace(G) exceeds the
// subtracted term, so a completed factorisation proves s <= lambda_min(X^T X).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "engine.h"
#include "kernels.h"
#include "mixed.h"

namespace cgl {

void build_gram(int xtype, const void* xt, int64_t n_pad, int64_t n, int64_t p, double* G,
                int64_t ldg, double* part, size_t cap, hipStream_t s) {
  CGL_HIP(hipMemsetAsync(G, 0, (size_t)p * ldg * 8, s));
  const size_t esz = xtype == XT_F64 ? 8 : (xtype == XT_F32 ? 4 : 2);
  const int64_t rows = 256;
  DevBuf wide;
  wide.alloc((size_t)rows * n_pad * 8);
  for (int64_t j0 = 0; j0 < p; j0 += rows) {  // G rows j0 .. j0 + r
    const int64_t r = std::min(rows, p - j0);
    launch_widen(xtype, (const char*)xt + (size_t)j0 * n_pad * esz, n_pad, r, n_pad,
                 wide.as<double>(), n_pad, s);
    launch_gemm_f64(xtype, xt, n_pad, p, n, wide.as<double>(), n_pad, (int)r, G + j0 * ldg, ldg,
                    part, cap, s);
  }
  CGL_HIP(hipStreamSynchronize(s));  // the staging rows are released here
}

namespace {

struct GramCheck {
  DevBuf G, work, fail;
  int64_t ldg = 0;
  double margin = 0.0;  // delta above
};

void gram_for_check(Problem& P, GramCheck& C) {
  hipStream_t s = P.ctx->stream;
  const int64_t n_pad = (P.n + 255) / 256 * 256;
  DevBuf xt, part;
  xt.alloc((size_t)P.p * n_pad * (P.xtype == XT_F64 ? 8 : (P.xtype == XT_F32 ? 4 : 2)));
  launch_transpose(P.xtype, P.X.ptr, P.ldx, P.n, P.p, n_pad, xt.ptr, s);
  C.ldg = (P.p + 255) / 256 * 256;
  C.G.alloc((size_t)P.p * C.ldg * 8);
  const size_t cap = 4 * (size_t)256 * (size_t)C.ldg * 8;
  part.alloc(cap);
  build_gram(P.xtype, xt.ptr, n_pad, P.n, P.p, C.G.as<double>(), C.ldg, part.as<double>(), cap, s);
  std::vector<double> diag((size_t)P.p);
  CGL_HIP(hipMemcpy2D(diag.data(), 8, C.G.ptr, (size_t)(C.ldg + 1) * 8, 8, (size_t)P.p,
                      hipMemcpyDeviceToHost));
  double tr = 0.0;
  for (double d : diag) tr += d;
  const double u = std::ldexp(1.0, -53);
  C.margin = 4.0 * (double)(P.n + P.p + 2) * u * tr;
  C.work.alloc(C.G.bytes);
  C.fail.alloc(sizeof(int));
}

bool factor_ok(Problem& P, GramCheck& C, double shift) {
  hipStream_t s = P.ctx->stream;
  CGL_HIP(hipMemcpyAsync(C.work.ptr, C.G.ptr, C.G.bytes, hipMemcpyDeviceToDevice, s));
  CGL_HIP(hipMemsetAsync(C.fail.ptr, 0, sizeof(int), s));
  launch_chol_factor(C.work.as<double>(), C.ldg, P.p, shift + C.margin, C.fail.as<int>(), s);
  CGL_HIP(hipGetLastError());
  int fail = 1;
  CGL_HIP(hipMemcpyAsync(&fail, C.fail.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  CGL_HIP(hipStreamSynchronize(s));
  return fail == 0;
}

}  // namespace

bool eigen_shift_proved(Problem& P, double shift) {
  if (shift == 0.0) return true;  // X^T X is positive semidefinite
  if (P.n < P.p) return false;    // X^T X is singular: lambda_min = 0
  GramCheck C;
  gram_for_check(P, C);
  return factor_ok(P, C, shift);
}

double eigen_shift_certified(Problem& P, double rel_tol) {
  if (P.n < P.p) return 0.0;
  GramCheck C;
  gram_for_check(P, C);
  // bisection on the shift: lo proved (0 needs no proof), hi above lambda_max or not proved
  double lo = 0.0, hi = P.lam_max > 0.0 ? 1.01 * P.lam_max : 0.0;
  if (hi <= 0.0) {
    std::vector<double> diag((size_t)P.p);
    CGL_HIP(hipMemcpy2D(diag.data(), 8, C.G.ptr, (size_t)(C.ldg + 1) * 8, 8, (size_t)P.p,
                        hipMemcpyDeviceToHost));
    hi = *std::max_element(diag.begin(), diag.end());  // lambda_min <= min_j G_jj <= max_j G_jj
  }
  // to a width of rel_tol relative to the proved shift once there is one
  for (int it = 0; it < 80 && hi - lo > rel_tol * (lo > 0.0 ? lo : hi); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (factor_ok(P, C, mid)) lo = mid;
    else hi = mid;
  }
  return lo;
}

}  // namespace cgl

// Host-side argument checks of the C ABI, exercised without a GPU: every call here must return
// CGL_E_INVAL (or the documented value) before touching a device. Built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of the library and of this driver; any sanitizer
// report aborts the run. Prints one line per failed expectation and exits with their count.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/certglm.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL: %s (last error: %s)\n", what, cgl_last_error());
    ++failures;
  }
}

static void expect_inval(int st, const char* what) {
  expect(st == CGL_E_INVAL && std::strlen(cgl_last_error()) > 0, what);
}

int main() {
  expect(cgl_version() == CGL_ABI_VERSION, "version");
  for (int s = 0; s <= 7; ++s) expect(cgl_status_str(s) != nullptr, "status string");
  cgl_node nd;
  cgl_node_init(&nd);
  expect(nd.tol == 1e-6 && nd.max_iter == 100000 && std::isinf(nd.incumbent), "node defaults");
  cgl_node_init(nullptr);

  // ---- node validation (host only)
  const int64_t p = 10;
  const int32_t k = 3;
  int32_t inf = -1;
  expect(cgl_node_validate(&nd, p, k, &inf) == CGL_OK && inf == 0, "default node valid");
  expect_inval(cgl_node_validate(nullptr, p, k, &inf), "NULL node");
  expect_inval(cgl_node_validate(&nd, 0, k, &inf), "p < 1");
  expect_inval(cgl_node_validate(&nd, p, 0, &inf), "k < 1");
  const int32_t dup[2] = {2, 2}, out[1] = {10}, neg[1] = {-1}, z[2] = {1, 4}, o[2] = {4, 5};
  cgl_node a = nd;
  a.fixed_zero = dup; a.n_zero = 2;
  expect_inval(cgl_node_validate(&a, p, k, &inf), "duplicate fixed_zero");
  a = nd; a.fixed_zero = out; a.n_zero = 1;
  expect_inval(cgl_node_validate(&a, p, k, &inf), "fixed_zero out of range");
  a = nd; a.fixed_in = neg; a.n_in = 1;
  expect_inval(cgl_node_validate(&a, p, k, &inf), "negative fixed_in");
  a = nd; a.fixed_zero = z; a.n_zero = 2; a.fixed_in = o; a.n_in = 2;
  expect_inval(cgl_node_validate(&a, p, k, &inf), "overlapping Z0 and Z1");
  a = nd; a.n_zero = 3; a.fixed_zero = nullptr;
  expect_inval(cgl_node_validate(&a, p, k, &inf), "NULL fixed_zero with n_zero > 0");
  a = nd; a.n_in = -1;
  expect_inval(cgl_node_validate(&a, p, k, &inf), "negative n_in");
  a = nd; a.tol = std::nan("");
  expect_inval(cgl_node_validate(&a, p, k, &inf), "NaN tol");
  a = nd; a.max_iter = 0;
  expect_inval(cgl_node_validate(&a, p, k, &inf), "max_iter 0");
  a = nd; a.check_every = 0;
  expect_inval(cgl_node_validate(&a, p, k, &inf), "check_every 0");
  a = nd; a.precision = 7;
  expect_inval(cgl_node_validate(&a, p, k, &inf), "unknown precision");
  a = nd; a.incumbent = std::nan("");
  expect_inval(cgl_node_validate(&a, p, k, &inf), "NaN incumbent");
  std::vector<double> ws((size_t)p, 0.5);
  ws[3] = std::numeric_limits<double>::infinity();
  a = nd; a.warm_start = ws.data();
  expect_inval(cgl_node_validate(&a, p, k, &inf), "non-finite warm start");
  const int32_t many[4] = {0, 1, 2, 3};
  a = nd; a.fixed_in = many; a.n_in = 4;
  expect(cgl_node_validate(&a, p, k, &inf) == CGL_OK && inf == 1, "|Z1| > k is infeasible");

  // ---- problem creation: argument checks before any device work
  const int64_t n = 6;
  std::vector<double> X((size_t)(n * p), 0.25), y((size_t)n, 1.0);
  cgl_problem* prob = nullptr;
  auto create = [&](const void* Xp, int dt, int64_t nn, int64_t pp, int64_t ldx, const double* yp,
                    int loss, double l2, double M, int kk, double L) {
    return cgl_problem_create(nullptr, Xp, dt, CGL_MEM_HOST, nn, pp, ldx, yp, loss, l2, M, kk, L,
                              &prob);
  };
  expect_inval(create(X.data(), CGL_F64, n, p, p, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0),
               "NULL context (valid arguments otherwise)");
  expect_inval(cgl_problem_create(nullptr, X.data(), CGL_F64, CGL_MEM_HOST, n, p, p, y.data(),
                                  CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0, nullptr), "NULL out");
  expect_inval(create(nullptr, CGL_F64, n, p, p, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0), "NULL X");
  expect_inval(create(X.data(), CGL_F64, 0, p, p, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0), "n < 1");
  expect_inval(create(X.data(), CGL_F64, n, 40000, 40000, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0),
               "p > 32768");
  expect_inval(create(X.data(), CGL_F64, n, p, p - 1, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0), "ldx < p");
  expect_inval(create(X.data(), 9, n, p, p, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0), "bad dtype");
  expect_inval(create(X.data(), CGL_F64, n, p, p, y.data(), 11, 1e-3, 2.0, 3, 0.0), "bad loss");
  expect_inval(create(X.data(), CGL_F64, n, p, p, y.data(), CGL_LOSS_POISSON, 1e-3, 2.0, 3, 0.0),
               "Poisson without L");
  expect_inval(create(X.data(), CGL_F64, n, p, p, y.data(), CGL_LOSS_LS, 0.0, 2.0, 3, 0.0), "lambda2 0");
  expect_inval(create(X.data(), CGL_F64, n, p, p, y.data(), CGL_LOSS_LS, 1e-3, -1.0, 3, 0.0), "M < 0");
  expect_inval(create(X.data(), CGL_F64, n, p, p, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 0, 0.0), "k 0");
  std::vector<double> ybad = y;
  ybad[2] = std::nan("");
  expect_inval(create(X.data(), CGL_F64, n, p, p, ybad.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0), "NaN y");
  ybad = y;
  ybad[1] = 0.5;
  expect_inval(create(X.data(), CGL_F64, n, p, p, ybad.data(), CGL_LOSS_LOGISTIC, 1e-3, 2.0, 3, 0.0),
               "logistic label 0.5");
  ybad[1] = -2.0;
  expect_inval(create(X.data(), CGL_F64, n, p, p, ybad.data(), CGL_LOSS_POISSON, 1e-3, 2.0, 3, 1.0),
               "negative Poisson response");
  ybad[1] = 0.0;
  expect_inval(create(X.data(), CGL_F64, n, p, p, ybad.data(), CGL_LOSS_GAMMA, 1e-3, 2.0, 3, 1.0),
               "zero Gamma response");
  std::vector<double> Xbad = X;
  Xbad[17] = std::numeric_limits<double>::infinity();
  expect_inval(create(Xbad.data(), CGL_F64, n, p, p, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0),
               "infinite entry of a host FP64 X");
  std::vector<float> Xf((size_t)(n * p), 0.5f);
  Xf[3] = std::nanf("");
  expect_inval(create(Xf.data(), CGL_F32, n, p, p, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0),
               "NaN entry of a host FP32 X");
  std::vector<uint16_t> Xh((size_t)(n * p), 0x3f80);  // BF16 1.0
  Xh[5] = 0x7f80;                                      // BF16 +infinity
  expect_inval(create(Xh.data(), CGL_BF16, n, p, p, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0),
               "infinite entry of a host BF16 X");
  // padded rows (ldx > p): the padding is not part of X and may hold anything
  std::vector<double> Xp((size_t)(n * (p + 2)), 1.0);
  for (int64_t i = 0; i < n; ++i) Xp[(size_t)(i * (p + 2) + p)] = std::nan("");
  expect_inval(create(Xp.data(), CGL_F64, n, p, p + 2, y.data(), CGL_LOSS_LS, 1e-3, 2.0, 3, 0.0),
               "padded X reaches the context check");
  expect(std::strstr(cgl_last_error(), "ctx") != nullptr, "padding is not scanned");

  // ---- entry points that need a context or objects refuse NULL without touching a device
  cgl_result res;
  expect_inval(cgl_solve_node(nullptr, &nd, nullptr, &res), "solve without problem");
  expect_inval(cgl_solve_batch(nullptr, &nd, 1, nullptr, &res), "batch without problem");
  expect_inval(cgl_prox_node_batch(nullptr, 1.0, 1.0, 3, nullptr, X.data(), 1, p, X.data(), nullptr),
               "prox without context");
  expect_inval(cgl_prox_batch_noalloc(nullptr, 1.0, 1.0, 3, X.data(), 1, p, X.data(), nullptr),
               "allocation-free prox without context");
  expect_inval(cgl_server_create(nullptr, 0, 256, nullptr), "server without out");
  expect(cgl_problem_destroy(nullptr) == CGL_OK && cgl_ctx_destroy(nullptr) == CGL_OK &&
             cgl_server_destroy(nullptr) == CGL_OK, "destroying NULL is a no-op");
  std::printf("%d failed\n", failures);
  return failures;
}

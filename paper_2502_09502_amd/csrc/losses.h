// Elementwise GLM losses f_i(u) of problem (1), their derivatives, and the conjugate terms of the
// weak-duality bound at zeta = -grad f (App. D.1), in FP64. Shared by the plain and the batched
// kernels; the host uses the constants at the end.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "solver.h"

namespace cgl {

__device__ __forceinline__ double softplus(double t) {
  return t > 0.0 ? t + log1p(exp(-t)) : log1p(exp(t));
}
__device__ __forceinline__ double sigmoid(double t) {
  if (t >= 0.0) return 1.0 / (1.0 + exp(-t));
  const double e = exp(t);
  return e / (1.0 + e);
}

// h(z) = z log z - z (z > 0), h(0) = 0 (App. D.1)
__device__ __forceinline__ double xlogx_minus_x(double z) {
  return z > 0.0 ? z * log(z) - z : 0.0;
}

// f_i(u)
__device__ __forceinline__ double loss_val(int loss, double u, double y) {
  if (loss == LOSS_LS) {
    const double r = u - y;
    return r * r;
  }
  if (loss == LOSS_POISSON) return exp(u) - y * u;
  if (loss == LOSS_GAMMA) return y * exp(-u) + u;
  if (loss == LOSS_SQHINGE) {
    const double m = fmax(0.0, 1.0 - y * u);
    return m * m;
  }
  return softplus(-y * u);
}

// d f_i / du
__device__ __forceinline__ double loss_grad(int loss, double u, double y) {
  if (loss == LOSS_LS) return 2.0 * (u - y);
  if (loss == LOSS_SQHINGE) return -2.0 * y * fmax(0.0, 1.0 - y * u);
  if (loss == LOSS_POISSON) return exp(u) - y;
  if (loss == LOSS_GAMMA) return 1.0 - y * exp(-u);
  return -y * sigmoid(-y * u);
}

// F_i*(-zeta_i) at zeta_i = -d f_i/du (u):
//   least squares  1/4 zeta^2 - y zeta;
//   logistic       q log q + (1 - q) log(1 - q), q = y zeta = sigmoid(-y u) (written with softplus);
//   squared hinge  h(-y zeta) with h(z) = z + z^2/4, -y zeta = -2 max(0, 1 - y u) <= 0;
//   Poisson        h(y - zeta) with h(z) = z log z - z, y - zeta = exp(u);
//   Gamma          y h((1 + zeta) / y) (the conjugate of y exp(-u) + u), (1 + zeta) / y = exp(-u).
__device__ __forceinline__ double fstar_term(int loss, double u, double y) {
  if (loss == LOSS_POISSON) return xlogx_minus_x(exp(u));
  if (loss == LOSS_GAMMA) return y * xlogx_minus_x(exp(-u));
  if (loss == LOSS_LS) {
    const double z = -2.0 * (u - y);
    return 0.25 * z * z - y * z;
  }
  if (loss == LOSS_SQHINGE) {
    const double m = fmax(0.0, 1.0 - y * u);
    return m * m - 2.0 * m;
  }
  const double t = -y * u;
  const double q = sigmoid(t);
  return -q * softplus(-t) - (1.0 - q) * softplus(t);
}

// Host constants. Lipschitz constant of d f_i/du (L = factor * lambda_max(X^T X)); 0 when there
// is none (Poisson, Gamma: the caller supplies L). At u = 0: d f_i/du = grad0_a + grad0_b * y_i
// and f_i(0).
inline double loss_lipschitz_factor(int loss) {
  if (loss == LOSS_LOGISTIC) return 0.25;
  if (loss == LOSS_POISSON || loss == LOSS_GAMMA) return 0.0;
  return 2.0;
}
inline double loss_grad0_a(int loss) {
  return (loss == LOSS_POISSON || loss == LOSS_GAMMA) ? 1.0 : 0.0;
}
inline double loss_grad0_b(int loss) {
  if (loss == LOSS_LOGISTIC) return -0.5;
  if (loss == LOSS_POISSON || loss == LOSS_GAMMA) return -1.0;
  return -2.0;
}
inline double loss_at0(int loss, double y) {
  if (loss == LOSS_LS) return y * y;
  if (loss == LOSS_SQHINGE || loss == LOSS_POISSON) return 1.0;
  if (loss == LOSS_GAMMA) return y;
  return std::log(2.0);
}

}  // namespace cgl

// FP64 Cholesky test of a symmetric matrix on the device: does the factorisation A = L L^T of
// A - shift I run to completion with positive pivots? Used to prove a lower bound on
// lambda_min(X^T X) for the eigen-perspective relaxation (App. D.2), where Q = X^T X - s I must
// be positive semidefinite.
//
// Right-looking, in panels of 64 columns; only the lower triangle is read. Per panel j0:
//   k_chol_diag   factors the 64 x 64 diagonal block in LDS (one workgroup);
//   k_chol_panel  L21 = A21 L11^{-T}, one thread per row (forward substitution, L11 in LDS);
//   k_chol_update A22 -= L21 L21^T on the 64 x 64 tiles of the lower triangle.
// A non-positive (or non-finite) pivot sets *fail; every later kernel returns at once.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "kernels.h"

namespace cgl {

constexpr int CB = 64;  // panel width

__global__ void k_shift_diag(double* __restrict__ A, int64_t lda, int64_t p, double shift) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < p) A[j * lda + j] -= shift;
}

__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ A, int64_t lda, int64_t p,
                                                   int64_t j0, int* __restrict__ fail) {
  __shared__ double T[CB][CB + 1];
  __shared__ int bad;
  if (*fail) return;
  const int tid = threadIdx.x;
  const int nb = (int)min((int64_t)CB, p - j0);
  for (int e = tid; e < nb * nb; e += blockDim.x) {
    const int r = e / nb, c = e % nb;
    T[r][c] = c <= r ? A[(j0 + r) * lda + j0 + c] : 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    if (tid == 0) {
      const double d = T[c][c];
      if (!(d > 0.0) || !isfinite(d)) bad = 1;
      else T[c][c] = sqrt(d);
    }
    __syncthreads();
    if (bad) break;
    const double piv = T[c][c];
    for (int r = c + 1 + tid; r < nb; r += blockDim.x) T[r][c] /= piv;
    __syncthreads();
    // trailing part of the block: T[r][q] -= T[r][c] T[q][c], c < q <= r
    const int m = nb - c - 1;
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int r = c + 1 + e / m, q = c + 1 + e % m;
      if (q <= r) T[r][q] -= T[r][c] * T[q][c];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) *fail = 1;
    return;
  }
  for (int e = tid; e < nb * nb; e += blockDim.x) {
    const int r = e / nb, c = e % nb;
    if (c <= r) A[(j0 + r) * lda + j0 + c] = T[r][c];
  }
}

// rows i >= j0 + CB: x L11^T = a (a = A[i][j0 .. j0 + CB)), overwritten by x
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ A, int64_t lda, int64_t p,
                                                    int64_t j0, const int* __restrict__ fail) {
  __shared__ double Lt[CB][CB + 1];
  if (*fail) return;
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e / CB, c = e % CB;
    Lt[r][c] = c <= r ? A[(j0 + r) * lda + j0 + c] : 0.0;
  }
  __syncthreads();
  const int64_t i = j0 + CB + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p) return;
  double* a = A + i * lda + j0;
  double x[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) x[c] = a[c];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    double s = x[c];
#pragma unroll
    for (int k = 0; k < c; ++k) s -= x[k] * Lt[c][k];
    x[c] = s / Lt[c][c];
  }
#pragma unroll
  for (int c = 0; c < CB; ++c) a[c] = x[c];
}

// A[i][j] -= sum_c L[i][c] L[j][c] for j <= i (tile granularity), i, j >= j1 = j0 + CB, where
// L[i][c] = A[i][j0 + c]. Tile t of the lower triangle: (ti, tj), tj <= ti, t = ti (ti + 1) / 2 + tj.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ A, int64_t lda, int64_t p,
                                                     int64_t j0, const int* __restrict__ fail) {
  __shared__ double Li[CB][CB / 2 + 1];
  __shared__ double Lj[CB][CB / 2 + 1];
  if (*fail) return;
  const int64_t t = blockIdx.x;
  int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int64_t tj = t - ti * (ti + 1) / 2;
  const int64_t j1 = j0 + CB;
  const int64_t i0 = j1 + ti * CB, c0 = j1 + tj * CB;
  const int tid = threadIdx.x;
  const int tr = (tid >> 4) * 4, tc = (tid & 15) * 4;  // 4 x 4 outputs per thread
  double acc[4][4] = {};
  for (int h = 0; h < CB; h += CB / 2) {
    __syncthreads();
    for (int e = tid; e < CB * (CB / 2); e += blockDim.x) {
      const int r = e / (CB / 2), c = e % (CB / 2);
      Li[r][c] = (i0 + r < p) ? A[(i0 + r) * lda + j0 + h + c] : 0.0;
      Lj[r][c] = (c0 + r < p) ? A[(c0 + r) * lda + j0 + h + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < CB / 2; ++c) {
      double ai[4], aj[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ai[q] = Li[tr + q][c];
        aj[q] = Lj[tc + q][c];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[q][r] += ai[q] * aj[r];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = i0 + tr + q;
    if (i >= p) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = c0 + tc + r;
      if (j < p && j <= i) A[i * lda + j] -= acc[q][r];
    }
  }
}

void launch_chol_factor(double* A, int64_t lda, int64_t p, double shift, int* fail,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_shift_diag, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, s, A, lda, p,
                     shift);
  for (int64_t j0 = 0; j0 < p; j0 += CB) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, A, lda, p, j0, fail);
    const int64_t rest = p - (j0 + CB);
    if (rest <= 0) break;
    hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, A,
                       lda, p, j0, (const int*)fail);
    const int64_t T = (rest + CB - 1) / CB;
    hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, s, A, lda,
                       p, j0, (const int*)fail);
  }
}

}  // namespace cgl

"""Seeded synthetic inputs: design matrices, labels, branch-and-bound node sets, arrival times.

This module holds none of the solver's arithmetic. It follows the synthetic generator of the
paper's experimental setup (App. B.2) with these readings:

* rows x_i iid N(0, Sigma) with Sigma_jl = 0.5^|j - l|, produced exactly by an AR(1) recursion
  along the columns: x_0 = e_0, x_j = 0.5 x_{j-1} + sqrt(0.75) e_j with e iid N(0, 1);
* every column centred and divided by its population standard deviation (so ||X_j||^2 = n);
* beta* has k ones at the 0-based positions m * (p // k) - 1, m = 1..k (the paper's
  "j mod (p/k) = 0" in 1-based indexing);
* least squares: y = X beta* + sigma * eps with sigma^2 = ||X beta*||^2 / (n * SNR), SNR = 5;
* logistic and squared hinge: y_i = +1 with probability sigmoid(x_i^T beta*), else -1;
* Poisson: counts with mean exp(x_i^T beta*); Gamma: shape-2 responses with that mean;
* lower-precision storage: FP32 = round-to-nearest-even of the FP64 values, BF16 = RNE of the
  FP32 values. When a problem is stored in FP32 or BF16, those rounded values ARE the problem.

Random streams: data uses ``default_rng([seed, config_id, p, loss_id])``; node sets use
``default_rng([1, config_id, p])``; arrivals use ``default_rng([2, config_id])``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LOSS_ID = {"ls": 0, "logistic": 1, "sqhinge": 2, "poisson": 3, "gamma": 4}


# ---------------------------------------------------------------------------------------------
# Precision helpers (storage formats only)
# ---------------------------------------------------------------------------------------------


def to_bf16_bits(x) -> np.ndarray:
    """Round FP32 values to bfloat16 (round to nearest, ties to even); return the 16-bit
    patterns as uint16. Inputs must be finite."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    bias = ((u >> 16) & 1) + 0x7FFF
    return ((u + bias) >> 16).astype(np.uint16)


def bf16_bits_to_f32(b) -> np.ndarray:
    """Exact widening of bfloat16 bit patterns to float32."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


# ---------------------------------------------------------------------------------------------
# Design matrix, coefficients, labels (App. B.2)
# ---------------------------------------------------------------------------------------------


def design_matrix(n: int, p: int, rng: np.random.Generator, corr: float = 0.5) -> np.ndarray:
    """Standardised Toeplitz-correlated Gaussian design, FP64, row-major n x p."""
    xt = rng.standard_normal((p, n))  # row j of xt is column j of X
    c = np.sqrt(1.0 - corr * corr)
    for j in range(1, p):
        xt[j] *= c
        xt[j] += corr * xt[j - 1]
    xt -= xt.mean(axis=1, keepdims=True)
    xt /= xt.std(axis=1, keepdims=True)
    return np.ascontiguousarray(xt.T)


def beta_star(p: int, k: int) -> np.ndarray:
    b = np.zeros(p)
    step = p // k
    b[np.arange(1, k + 1) * step - 1] = 1.0
    return b


def labels(X: np.ndarray, b_star: np.ndarray, loss: str, rng: np.random.Generator,
           snr: float = 5.0) -> np.ndarray:
    u = X @ b_star
    n = X.shape[0]
    if loss == "ls":
        sigma = np.sqrt(float(u @ u) / (n * snr))
        return u + sigma * rng.standard_normal(n)
    if loss in ("logistic", "sqhinge"):  # classification labels in {-1, +1}
        prob = 1.0 / (1.0 + np.exp(-u))
        return np.where(rng.random(n) < prob, 1.0, -1.0)
    if loss == "poisson":  # counts with mean exp(x_i^T beta*)
        return rng.poisson(np.exp(u)).astype(np.float64)
    if loss == "gamma":  # positive responses with mean exp(x_i^T beta*), shape 2
        return rng.gamma(2.0, np.exp(u) / 2.0)
    raise ValueError(loss)


@dataclass
class Dataset:
    """One synthetic problem. ``X`` holds the problem's values in FP64 (exact upcast of the stored
    format); ``X_store`` is the stored array (float64, float32, or uint16 bfloat16 patterns)."""

    name: str
    n: int
    p: int
    k: int
    M: float
    lam2: float
    loss: str
    dtype: str  # "f64", "f32" or "bf16"
    X: np.ndarray
    X_store: np.ndarray
    y: np.ndarray
    beta_star: np.ndarray


def make_dataset(n, p, k, loss="ls", dtype="f64", M=2.0, lam2=1e-3, seed=0, config_id=0,
                 k_true=None, name="") -> Dataset:
    k_true = k if k_true is None else k_true
    rng = np.random.default_rng([seed, config_id, p, LOSS_ID[loss]])
    X64 = design_matrix(n, p, rng)
    bs = beta_star(p, k_true)
    y = labels(X64, bs, loss, rng)
    if dtype == "f64":
        X_store = X64
        X = X64
    elif dtype == "f32":
        X_store = X64.astype(np.float32)
        X = X_store.astype(np.float64)
    elif dtype == "bf16":
        X_store = to_bf16_bits(X64.astype(np.float32))
        X = bf16_bits_to_f32(X_store).astype(np.float64)
    else:
        raise ValueError(dtype)
    return Dataset(name=name, n=n, p=p, k=k, M=M, lam2=lam2, loss=loss, dtype=dtype, X=X,
                   X_store=X_store, y=y, beta_star=bs)


# ---------------------------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------------------------

CONFIGS = {
    # least-squares root relaxation, plain FP64, tiny
    "c1": dict(n=200, p=50, k=5, loss="ls", dtype="f64", config_id=1),
    # least-squares root relaxation, single iterate, HBM-bound GEMV path
    "c2_f64": dict(n=10000, p=5000, k=10, loss="ls", dtype="f64", config_id=2),
    "c2_f32": dict(n=10000, p=5000, k=10, loss="ls", dtype="f32", config_id=2),
    # logistic root relaxation, FP32 design
    "c3": dict(n=20000, p=10000, k=10, loss="logistic", dtype="f32", config_id=3),
    # 256 least-squares nodes sharing one BF16 design
    "c4": dict(n=20000, p=10000, k=10, loss="ls", dtype="bf16", config_id=4),
}


def make_config(name: str, seed: int = 0, **overrides) -> Dataset:
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    return make_dataset(seed=seed, name=name, **cfg)


def serving_dataset(p: int, k: int = 10, seed: int = 0, config_id: int = 5):
    """One resident dataset of the serving workload: n = 2p, FP32 design, and two label vectors
    (least squares, logistic) drawn from the same design. Returns (X_f32, y_ls, y_logistic)."""
    n = 2 * p
    rng = np.random.default_rng([seed, config_id, p, LOSS_ID["ls"]])
    X64 = design_matrix(n, p, rng)
    bs = beta_star(p, k)
    y_ls = labels(X64, bs, "ls", rng)
    y_log = labels(X64, bs, "logistic", np.random.default_rng([seed, config_id, p, LOSS_ID["logistic"]]))
    X32 = X64.astype(np.float32)
    del X64
    return X32, y_ls, y_log


def node_sets(p: int, k: int, count: int, zero_cap: int, seed: int = 1, config_id: int = 0):
    """Branch-and-bound node sets: |Z0| ~ U{0..zero_cap}, |Z1| ~ U{0..min(zero_cap, k)}, disjoint
    uniform-random index subsets (sorted, 0-based)."""
    rng = np.random.default_rng([seed, config_id, p])
    out = []
    for _ in range(count):
        a = int(rng.integers(0, zero_cap + 1))
        b = int(rng.integers(0, min(zero_cap, k) + 1))
        perm = rng.permutation(p)
        out.append((np.sort(perm[:a]).astype(np.int32), np.sort(perm[a:a + b]).astype(np.int32)))
    return out


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 2, config_id: int = 5):
    """Arrival times (seconds from 0) with exponential inter-arrival gaps of mean 1 / rate."""
    rng = np.random.default_rng([seed, config_id])
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))

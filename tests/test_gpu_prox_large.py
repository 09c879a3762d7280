"""The device prox beyond p = 16384 (the long-vector kernel that streams each vector from
memory), element by element against the oracle's stack PAVA (Alg. 1 via the Moreau identity) and
g by Alg. 2, at the sizes of the standalone prox workload of Sec. 4.1 (p = 100 * 2^i up to
102400, gamma ~ N(0, I), k = 10, M = 1, rho = 1), from just past the switch away from the
register-held kernels at p = 16384, and around them: other k (both the candidate ranking and the
radix fallback), fixed sets, ties and zeros."""
import numpy as np
import pytest

import oracle
from paper_2502_09502_amd import _lib

from gpu_util import ctx

pytestmark = pytest.mark.gpu


def _check(W, rho, M, k, sets=None, atol=1e-11):
    beta, g = _lib.prox_node_batch(ctx(), W, rho, M, k, sets)
    for i in range(W.shape[0]):
        z0, z1 = sets[i] if sets is not None else ((), ())
        ns = oracle.node_sets(W.shape[1], z0, z1)
        ref = oracle.prox_node(W[i], rho, M, k, ns)
        scale = max(1.0, float(np.max(np.abs(W[i]))))
        err = float(np.max(np.abs(beta[i] - ref)))
        assert err <= atol * scale, (i, err)
        gref = oracle.g_node(ref, M, k, ns, slack=1e-9)
        assert abs(g[i] - gref) <= 1e-10 * max(1.0, abs(gref)), (i, g[i], gref)


@pytest.mark.parametrize("p", [16385, 25600, 32769, 51200, 102400])
def test_prox_fig1_setting_large_p(p):
    W = np.stack([np.random.default_rng([4, p, s]).standard_normal(p) for s in range(3)])
    _check(W, 1.0, 1.0, 10)


@pytest.mark.parametrize("k", [1, 63, 64, 256])
def test_prox_large_p_other_budgets(k):
    p = 40000
    rng = np.random.default_rng(k)
    W = rng.normal(0, 1, size=(2, p)) * np.array([[0.2], [4.0]])
    for rho, M in ((0.7, 0.5), (30.0, 2.0)):
        _check(W, rho, M, k)


def test_prox_large_p_ties_zeros_and_fixed_sets():
    p = 50000
    r = np.random.default_rng(7).normal(size=p)
    rows = [np.zeros(p), np.full(p, -0.5), np.round(r, 1)]
    sparse = np.zeros(p)
    sparse[::4999] = np.arange(1, 12)  # 11 nonzeros: k' beyond the nonzeros leaves zero ties
    rows.append(sparse)
    W = np.stack(rows)
    for k in (3, 10, 200):
        _check(W, 1.0, 2.0, k)
    rng = np.random.default_rng(9)
    sets = []
    for _ in range(W.shape[0]):
        idx = rng.permutation(p)
        sets.append((idx[:30].tolist(), idx[30:36].tolist()))
    _check(W, 2.0, 1.0, 10, sets)
    # budget used up by Z1 (k' = 0) and k' >= |F|
    sets0 = [((), list(range(10)))] * W.shape[0]
    _check(W, 1.0, 1.0, 10, sets0)
    _check(W[:2], 1.0, 1.0, 10, [(list(range(p - 5)), [])] * 2)

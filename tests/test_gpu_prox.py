"""GPU prox kernel (radix head select + tail root search) against the oracle's stack PAVA and
Alg. 2, element by element, through the C-ABI."""
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
        if len(z1) > k:
            continue
        ref = oracle.prox_node(W[i], rho, M, k, ns)
        scale = max(1.0, float(np.max(np.abs(W[i]))))
        err = float(np.max(np.abs(beta[i] - ref)))
        assert err <= atol * scale, (i, err)
        gref = oracle.g_node(ref, M, k, ns, slack=1e-9)
        assert abs(g[i] - gref) <= 1e-10 * max(1.0, abs(gref)), (i, g[i], gref)


@pytest.mark.parametrize("p", [1, 2, 7, 64, 1000, 1024, 1025, 3000, 5000, 8193, 10000, 10240, 20000])
@pytest.mark.parametrize("k", [1, 5, 10, 40])
def test_prox_random(p, k):
    rng = np.random.default_rng(p * 100 + k)
    W = rng.normal(0, 1, size=(3, p)) * np.array([[0.1], [1.0], [5.0]])
    for rho in (0.7, 30.0, 5e7):
        for M in (0.5, 2.0):
            _check(W, rho, M, k)


def test_prox_ties_zeros_and_constant_vectors():
    p = 3000
    rows = [np.zeros(p), np.full(p, 0.25), np.full(p, -3.0)]
    r = np.random.default_rng(1).normal(size=p)
    t = r.copy(); t[::3] = t[0]
    rows += [t, np.round(r, 1), np.where(np.arange(p) % 2 == 0, 1.0, -1.0)]
    W = np.stack(rows)
    for k in (1, 3, 10, 256, 3000, 5000):
        for rho in (1.0, 1e4):
            _check(W, rho, 2.0, k)


def test_prox_node_sets():
    rng = np.random.default_rng(7)
    p, k = 5000, 10
    W = rng.normal(size=(16, p))
    sets = []
    for i in range(16):
        perm = rng.permutation(p)
        a, b = int(rng.integers(0, 30)), int(rng.integers(0, 11))
        sets.append((perm[:a], perm[a:a + b]))
    sets[0] = ((), np.arange(10))          # k' = 0
    sets[1] = (np.arange(p - 5), ())       # |F| = 5 < k
    sets[2] = ((), np.arange(11))          # infeasible (skipped by the checker)
    _check(W, 3.0, 1.0, k, sets)
    _check(W, 4e6, 2.0, k, sets)


def test_prox_rejects_head_beyond_capacity():
    W = np.zeros((1, 3000))
    with pytest.raises(_lib.CglError):
        _lib.prox_node_batch(ctx(), W, 1.0, 1.0, 257)


@pytest.mark.parametrize("p", [100, 800, 6400, 25600])
def test_prox_standalone_workload_distribution(p):
    """The standalone prox workload's inputs (Fig. 1 setting: gamma ~ N(0, I_p), k = 10, M = 1,
    rho = 1), five seeds per size, element by element against the oracle."""
    W = np.stack([np.random.default_rng([4, p, s]).standard_normal(p) for s in range(5)])
    _check(W, 1.0, 1.0, 10)

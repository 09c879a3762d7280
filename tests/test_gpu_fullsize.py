"""Full-size parity of the paths the benchmark and serving workloads run, against the oracle.

* logistic root relaxation at n = 20000, p = 10000 with an FP32 design (App. D.1 logistic), on
  the plain FP64 path and on the batched mixed-precision engine;
* the 256-node workload's design (n = 20000, p = 10000, BF16): every bound the batched engine
  reports is re-evaluated by the oracle from the iterate that produced it (Sec. 3.4, weak
  duality: then the bound is valid whatever the iterate), and two nodes are checked against the
  oracle's own optimum solved to a 1e-9 gap;
* the largest serving design (n = 40000, p = 20000, FP32, least squares and logistic), where the
  node kernels keep 24 values per thread, through the request server and through batched solves.
"""
import functools

import numpy as np
import pytest

import oracle
from paper_2502_09502_amd import _lib, synth

from gpu_util import ctx, rel

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=1)
def _c3():
    return synth.make_config("c3")


@functools.lru_cache(maxsize=1)
def _c4():
    return synth.make_config("c4")


@functools.lru_cache(maxsize=1)
def _serving20k():
    X32, y_ls, y_log = synth.serving_dataset(20000)
    return X32, X32.astype(np.float64), y_ls, y_log


def _oracle_check(X, y, loss, lam2, M, k, z0, z1, r, tol=1e-6):
    """The oracle's objective at the returned beta equals the reported primal value, the oracle's
    own duality gap at that beta is within the tolerance, and the reported bound lies below the
    oracle's objective there."""
    ns = oracle.node_sets(X.shape[1], z0, z1)
    P = oracle.primal_value(X, y, loss, lam2, M, k, ns, r.beta)
    zeta = -oracle.get_loss(loss).grad(X @ r.beta, y)
    D = oracle.dual_value(X, y, loss, lam2, M, k, ns, zeta)
    assert rel(P, r.primal) <= 1e-10, (P, r.primal)
    assert (P - D) / max(abs(P), 1.0) <= 2.0 * tol, (P, D)
    assert r.lower_bound <= P
    return P


def _witness_check(X, y, loss, lam2, M, k, z0, z1, r, dual_beta):
    """The reported bound is D(zeta) at zeta = -grad f(X beta_D) for the iterate beta_D the engine
    returned with it, re-evaluated by the oracle in FP64."""
    ns = oracle.node_sets(X.shape[1], z0, z1)
    zeta = -oracle.get_loss(loss).grad(X @ dual_beta, y)
    D = oracle.dual_value(X, y, loss, lam2, M, k, ns, zeta)
    assert abs(D - r.lower_bound) <= 1e-10 * max(abs(r.primal), 1.0), (D, r.lower_bound)
    assert np.all(dual_beta[ns.zero] == 0.0)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_config3_logistic_full_size(precision):
    d = _c3()
    prob = _lib.Problem(ctx(), d.X_store, d.y, loss="logistic", lam2=d.lam2, M=d.M, k=d.k)
    sets = [((), ())] + synth.node_sets(d.p, d.k, 3, 20, config_id=3)
    specs = [prob.node(Z0=z0, Z1=z1, tol=1e-6, max_iter=20000, precision=precision)
             for z0, z1 in sets]
    if precision == "mixed":
        res, duals = prob.solve_batch_dual(specs)
    else:
        res, duals = prob.solve_batch(specs), None
    for i, ((z0, z1), r) in enumerate(zip(sets, res)):
        assert r.status == "converged" and r.gap_rel <= 1e-6, r
        _oracle_check(d.X, d.y, "logistic", d.lam2, d.M, d.k, z0, z1, r)
        if duals is not None:
            _witness_check(d.X, d.y, "logistic", d.lam2, d.M, d.k, z0, z1, r, duals[i])


@pytest.mark.timeout(600)
def test_config4_bounds_reproduced_by_the_oracle():
    d = _c4()
    prob = _lib.Problem(ctx(), d.X_store, d.y, loss="ls", lam2=d.lam2, M=d.M, k=d.k)
    sets = synth.node_sets(d.p, d.k, 16, 20, config_id=4)
    res, duals = prob.solve_batch_dual(
        [prob.node(Z0=z0, Z1=z1, tol=1e-6, precision="mixed") for z0, z1 in sets])
    for i, ((z0, z1), r) in enumerate(zip(sets, res)):
        assert r.status == "converged" and r.gap_rel <= 1e-6, r
        _oracle_check(d.X, d.y, "ls", d.lam2, d.M, d.k, z0, z1, r)
        _witness_check(d.X, d.y, "ls", d.lam2, d.M, d.k, z0, z1, r, duals[i])


@pytest.mark.timeout(900)
def test_config4_against_oracle_optimum():
    """Two nodes of the workload: the oracle's own solve to a 1e-9 gap bounds the GPU's bound from
    above, and the GPU's objective is within 1e-6 of the oracle's."""
    d = _c4()
    prob = _lib.Problem(ctx(), d.X_store, d.y, loss="ls", lam2=d.lam2, M=d.M, k=d.k)
    sets = synth.node_sets(d.p, d.k, 2, 20, config_id=4)
    res = prob.solve_batch([prob.node(Z0=z0, Z1=z1, tol=1e-6, precision="mixed")
                            for z0, z1 in sets])
    for (z0, z1), r in zip(sets, res):
        ref = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, d.k, z0, z1, tol=1e-9)
        assert ref.status == "converged"
        assert r.status == "converged", r
        assert r.lower_bound <= ref.primal
        assert rel(r.primal, ref.primal) <= 1e-6, (r.primal, ref.primal)
        assert ref.lower_bound <= r.primal


@pytest.mark.timeout(900)
def test_serving_largest_design_through_the_server():
    """n = 40000, p = 20000 (24 values per thread in the node kernels): four least-squares and
    four logistic requests on one design through the server, each checked against the oracle."""
    X32, X, y_ls, y_log = _serving20k()
    p = X.shape[1]
    probs = {loss: _lib.Problem(ctx(), X32, y, loss=loss, lam2=1e-3, M=2.0, k=10)
             for loss, y in (("ls", y_ls), ("logistic", y_log))}
    ys = {"ls": y_ls, "logistic": y_log}
    sets = synth.node_sets(p, 10, 8, 30, config_id=5)
    srv = _lib.Server(ctx(), 0, 256)
    jobs = {}
    for i, (z0, z1) in enumerate(sets):
        loss = "ls" if i % 2 == 0 else "logistic"
        spec = probs[loss].node(Z0=z0, Z1=z1, tol=1e-6, max_iter=5000, precision="mixed")
        jobs[srv.submit(probs[loss], spec)] = (loss, z0, z1)
    out = {}
    for _ in range(20000):
        for t, r, _lat in srv.poll(64):
            out[t] = r
        if len(out) == len(jobs):
            break
    srv.close()
    assert len(out) == len(jobs)
    for t, (loss, z0, z1) in jobs.items():
        r = out[t]
        assert r.status == "converged" and r.gap_rel <= 1e-6, (loss, r)
        _oracle_check(X, ys[loss], loss, 1e-3, 2.0, 10, z0, z1, r)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("loss", ["ls", "logistic"])
def test_serving_largest_design_bound_witnesses(loss):
    X32, X, y_ls, y_log = _serving20k()
    y = y_ls if loss == "ls" else y_log
    p = X.shape[1]
    prob = _lib.Problem(ctx(), X32, y, loss=loss, lam2=1e-3, M=2.0, k=10)
    sets = synth.node_sets(p, 10, 3, 30, config_id=6)
    res, duals = prob.solve_batch_dual(
        [prob.node(Z0=z0, Z1=z1, tol=1e-6, max_iter=5000, precision="mixed") for z0, z1 in sets])
    for i, ((z0, z1), r) in enumerate(zip(sets, res)):
        assert r.status == "converged" and r.gap_rel <= 1e-6, r
        _oracle_check(X, y, loss, 1e-3, 2.0, 10, z0, z1, r)
        _witness_check(X, y, loss, 1e-3, 2.0, 10, z0, z1, r, duals[i])

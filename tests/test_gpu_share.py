"""Problems on one design sharing a batched engine (cgl_problem_share_design): a least-squares
owner and a logistic sharer on the same X. Every node's result equals the one it gets on an
engine of its own (within the tolerance) and the oracle's certified optimum; a server serves
both problems' nodes from the owner's engine; the argument errors."""
import numpy as np
import pytest

import oracle
from paper_2502_09502_amd import _lib, synth

from gpu_util import ctx, rel

pytestmark = pytest.mark.gpu

P = 300
K = 10


def _data():
    X32, y_ls, y_log = synth.serving_dataset(P, K)
    return X32, y_ls, y_log


def _pair(X32, y_ls, y_log, share=True):
    a = _lib.Problem(ctx(), X32, y_ls, loss="ls", lam2=1e-3, M=2.0, k=K)
    b = _lib.Problem(ctx(), X32, y_log, loss="logistic", lam2=1e-3, M=2.0, k=K)
    if share:
        a.share_design(b)
    return a, b


def _specs(prob, sets):
    return [prob.node(Z0=z0, Z1=z1, tol=1e-6, max_iter=5000, precision="mixed") for z0, z1 in sets]


def _same(r, ref):
    assert r.status == "converged" and r.gap_rel <= 1e-6, r
    assert rel(r.primal, ref.primal) <= 2e-6, (r.primal, ref.primal)
    assert r.lower_bound <= ref.primal + 1e-9 * abs(ref.primal)
    assert ref.lower_bound <= r.primal + 1e-9 * abs(ref.primal)


def _oracle_check(X, y, loss, z0, z1, r):
    ref = oracle.solve_node(X, y, loss, 1e-3, 2.0, K, z0, z1, tol=1e-9)
    assert rel(r.primal, ref.primal) <= 1e-6, (r.primal, ref.primal)
    assert r.lower_bound <= ref.primal
    ns = oracle.node_sets(X.shape[1], z0, z1)
    Pb = oracle.primal_value(X, y, loss, 1e-3, 2.0, K, ns, r.beta)
    assert rel(Pb, r.primal) <= 1e-10


def test_shared_engine_batches_match_own_engines_and_oracle():
    X32, y_ls, y_log = _data()
    X = X32.astype(np.float64)
    a, b = _pair(X32, y_ls, y_log)
    a2, b2 = _pair(X32, y_ls, y_log, share=False)
    sets = synth.node_sets(P, K, 12, 20, config_id=91)
    # the sharer's nodes first (they build the owner's engine), then the owner's, then again
    rb = b.solve_batch(_specs(b, sets))
    ra = a.solve_batch(_specs(a, sets))
    rb_again = b.solve_batch(_specs(b, sets[:3]))
    ref_a = a2.solve_batch(_specs(a2, sets))
    ref_b = b2.solve_batch(_specs(b2, sets))
    for r, ref in zip(ra, ref_a):
        _same(r, ref)
    for r, ref in zip(rb, ref_b):
        _same(r, ref)
    for r, ref in zip(rb_again, ref_b[:3]):
        _same(r, ref)
    for i in (0, 5):
        _oracle_check(X, y_ls, "ls", *sets[i], ra[i])
        _oracle_check(X, y_log, "logistic", *sets[i], rb[i])


def test_server_serves_both_problems_from_one_engine():
    X32, y_ls, y_log = _data()
    X = X32.astype(np.float64)
    a, b = _pair(X32, y_ls, y_log)
    a2, b2 = _pair(X32, y_ls, y_log, share=False)
    sets = synth.node_sets(P, K, 20, 25, config_id=92)
    srv = _lib.Server(ctx(), 0, 256)
    jobs = []
    for i, (z0, z1) in enumerate(sets):
        prob, twin = (a, a2) if i % 2 == 0 else (b, b2)
        spec = prob.node(Z0=z0, Z1=z1, tol=1e-6, max_iter=5000, precision="mixed")
        jobs.append((srv.submit(prob, spec), twin, (z0, z1), prob is a))
    out = {}
    for _ in range(20000):
        for t, r, _lat in srv.poll(64):
            out[t] = r
        if len(out) == len(jobs):
            break
    assert len(out) == len(jobs), srv.stats()
    srv.close()
    for t, twin, (z0, z1), is_ls in jobs:
        ref = twin.solve_batch(_specs(twin, [(z0, z1)]))[0]
        _same(out[t], ref)
    t, _, (z0, z1), is_ls = jobs[3]
    _oracle_check(X, y_ls if is_ls else y_log, "ls" if is_ls else "logistic", z0, z1, out[t])


def test_share_design_errors_and_lifetimes():
    X32, y_ls, y_log = _data()
    a, b = _pair(X32, y_ls, y_log, share=False)
    with pytest.raises(_lib.CglError, match="own design"):
        a.share_design(a)
    other = X32.copy()
    other[3, 7] += 1.0
    c = _lib.Problem(ctx(), other, y_log, loss="logistic", lam2=1e-3, M=2.0, k=K)
    with pytest.raises(_lib.CglError, match="designs differ"):
        a.share_design(c)
    d = _lib.Problem(ctx(), X32[:, :200], y_ls, loss="ls", lam2=1e-3, M=2.0, k=K)
    with pytest.raises(_lib.CglError, match="differ in n, p"):
        a.share_design(d)
    a.share_design(b)
    with pytest.raises(_lib.CglError, match="already shares"):
        b.share_design(a)
    # the owner's engine exists after a mixed solve: no more sharers
    sets = synth.node_sets(P, K, 2, 10, config_id=93)
    a.solve_batch(_specs(a, sets))
    e = _lib.Problem(ctx(), X32, y_ls, loss="ls", lam2=2e-3, M=2.0, k=K)
    with pytest.raises(_lib.CglError, match="engine"):
        a.share_design(e)
    # a destroyed sharer leaves the owner's engine working; a destroyed owner leaves its sharer
    # standalone with an engine of its own
    b.close()
    r = a.solve_batch(_specs(a, sets))
    assert all(x.status == "converged" for x in r)
    f = _lib.Problem(ctx(), X32, y_log, loss="logistic", lam2=1e-3, M=2.0, k=K)
    g = _lib.Problem(ctx(), X32, y_ls, loss="ls", lam2=1e-3, M=2.0, k=K)
    g.share_design(f)
    g.close()
    r = f.solve_batch(_specs(f, sets))
    assert all(x.status == "converged" for x in r)

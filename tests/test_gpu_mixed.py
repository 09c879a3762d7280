"""Batched mixed-precision engine (BF16 MFMA corrections, FP64 re-centring and certificate)
against the oracle, and batched results against the same nodes solved alone."""
import math

import numpy as np
import pytest

import oracle
from paper_2502_09502_amd import _lib, synth

from gpu_util import ctx, rel

pytestmark = pytest.mark.gpu


def _problem(d):
    return _lib.Problem(ctx(), d.X_store, d.y, loss=d.loss, lam2=d.lam2, M=d.M, k=d.k)


def _specs(prob, sets, **kw):
    kw.setdefault("tol", 1e-6)
    kw.setdefault("max_iter", 5000)
    return [prob.node(Z0=z0, Z1=z1, precision="mixed", **kw) for z0, z1 in sets]


def _check(d, res, z0, z1, ref=None, tol=1e-6):
    ns = oracle.node_sets(d.p, z0, z1)
    if ref is None:
        ref = oracle.solve_node(d.X, d.y, d.loss, d.lam2, d.M, d.k, z0, z1, tol=1e-9)
    assert res.status == "converged", res
    assert res.gap_rel <= tol
    assert rel(res.primal, ref.primal) <= 1e-6, (res.primal, ref.primal)
    assert res.lower_bound <= ref.primal
    Pb = oracle.primal_value(d.X, d.y, d.loss, d.lam2, d.M, d.k, ns, res.beta)
    assert rel(Pb, res.primal) <= 1e-10


@pytest.mark.parametrize("loss", ["ls", "logistic", "sqhinge"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_small_batch_matches_oracle(loss, dtype):
    d = synth.make_dataset(500, 200, 8, loss=loss, dtype=dtype, config_id=80)
    prob = _problem(d)
    sets = synth.node_sets(d.p, d.k, 6, 12, config_id=80)
    res = prob.solve_batch(_specs(prob, sets))
    for (z0, z1), r in zip(sets, res):
        _check(d, r, z0, z1)


def test_repeated_recentring_to_tight_gap():
    """A tolerance far below the BF16 floor makes every node re-centre several times; a re-centre
    moves the base point under the running momentum (Alg. 3 restarts only on an objective
    increase), and the certified results still match the oracle."""
    d = synth.make_dataset(500, 200, 8, config_id=83)
    prob = _problem(d)
    sets = synth.node_sets(d.p, d.k, 6, 12, config_id=83)
    res = prob.solve_batch(_specs(prob, sets, tol=1e-8, max_iter=20000))
    assert max(r.recentres for r in res) >= 2
    for (z0, z1), r in zip(sets, res):
        _check(d, r, z0, z1, tol=1e-8)


def test_config1_mixed_root():
    d = synth.make_config("c1")
    prob = _problem(d)
    r = prob.solve(precision="mixed", tol=1e-6, max_iter=5000)
    _check(d, r, (), ())


def test_batched_equals_alone_and_refill():
    """More nodes than slots (continuous refill); each batched result equals the same node solved
    alone within the tolerance."""
    d = synth.make_dataset(400, 150, 6, config_id=81)
    prob = _problem(d)
    sets = synth.node_sets(d.p, d.k, 300, 15, config_id=81)
    batched = prob.solve_batch(_specs(prob, sets))
    assert all(r.status == "converged" and r.gap_rel <= 1e-6 for r in batched)
    for i in (0, 7, 150, 299):
        alone = prob.solve_batch(_specs(prob, [sets[i]]))[0]
        assert rel(batched[i].primal, alone.primal) <= 2e-6
        assert batched[i].lower_bound <= alone.primal + 1e-9 * abs(alone.primal)
        assert alone.lower_bound <= batched[i].primal + 1e-9 * abs(alone.primal)
    for i in (3, 250):
        _check(d, batched[i], *sets[i])


def test_refill_with_warm_starts_and_open_rounds():
    """More nodes than slots where the late nodes are warm-started: they are admitted into freed
    slots while certification rounds of other nodes are still queued, are parked until a round
    evaluates their start, and reach the oracle's certified optimum like cold nodes."""
    d = synth.make_dataset(400, 150, 6, config_id=83)
    prob = _problem(d)
    sets = synth.node_sets(d.p, d.k, 290, 15, config_id=83)
    rng = np.random.default_rng(83)
    specs = []
    for i, (z0, z1) in enumerate(sets):
        w = None
        if i >= 260:  # admitted only after earlier nodes retire
            w = 0.5 * rng.standard_normal(d.p) if i % 2 else np.zeros(d.p)
        specs.append(prob.node(Z0=z0, Z1=z1, tol=1e-6, max_iter=5000, precision="mixed",
                               warm_start=w))
    res = prob.solve_batch(specs)
    assert all(r.status == "converged" and r.gap_rel <= 1e-6 for r in res)
    for i in (1, 261, 262, 289):
        _check(d, res[i], *sets[i])


def test_mixed_edge_cases():
    d = synth.make_dataset(150, 40, 4, config_id=82)
    prob = _problem(d)
    specs = [
        prob.node(Z1=[0, 1, 2, 3, 4], precision="mixed"),             # infeasible
        prob.node(Z0=np.arange(40), precision="mixed"),               # everything fixed to 0
        prob.node(Z1=[3, 5, 7, 9], precision="mixed"),                # k' = 0
        prob.node(precision="mixed", max_iter=2),                     # cap
        prob.node(precision="mixed", max_iter=1),                     # no iteration at all
    ]
    r = prob.solve_batch(specs)
    assert r[0].status == "infeasible" and r[0].lower_bound == math.inf
    f0 = float(d.y @ d.y)
    assert r[1].status == "converged" and rel(r[1].primal, f0) < 1e-12
    ref = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, d.k, (), [3, 5, 7, 9], tol=1e-10)
    assert rel(r[2].primal, ref.primal) <= 1e-6 and r[2].lower_bound <= ref.primal
    root = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, d.k, tol=1e-10)
    for q in (3, 4):
        assert r[q].status == "not_converged" and r[q].lower_bound <= root.primal


def test_certification_round_with_empty_support():
    """A certification round whose iterates are all zero: the FP64 product X beta runs over an
    empty union of supports and must give u = 0 (P = f(0) = y'y for least squares)."""
    d = synth.make_dataset(150, 40, 4, config_id=82)
    prob = _problem(d)
    f0 = float(d.y @ d.y)
    r = prob.solve_batch([prob.node(Z0=np.arange(40), precision="mixed")])[0]
    assert r.status == "converged" and rel(r.primal, f0) < 1e-12
    assert np.all(r.beta == 0.0)
    r = prob.solve_batch([prob.node(precision="mixed", max_iter=1)])[0]
    root = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, d.k, tol=1e-10)
    assert r.status == "not_converged" and rel(r.primal, f0) < 1e-12
    assert r.lower_bound <= root.primal


def test_disjoint_supports_in_one_round():
    """Nodes whose free sets do not overlap are certified in the same rounds: the union of their
    supports covers coordinates that are zero for most of them, and each result still matches
    the oracle."""
    d = synth.make_dataset(400, 120, 5, config_id=84)
    prob = _problem(d)
    rng = np.random.default_rng(84)
    perm = rng.permutation(d.p)
    sets = [(np.sort(np.concatenate([perm[:40 * i], perm[40 * (i + 1):]])), np.array([], int))
            for i in range(3)]
    sets.append((np.array([], int), np.array([], int)))
    res = prob.solve_batch(_specs(prob, sets))
    for (z0, z1), r in zip(sets, res):
        assert np.all(r.beta[z0] == 0.0)
        _check(d, r, z0, z1)


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_gram_certificate_matches_direct_product(dtype, monkeypatch):
    """Least squares with n >= p certifies with X^T grad f(X beta) = 2 G beta - 2 X^T y from an
    FP64 Gram matrix; with the Gram matrix turned off the same nodes are certified by the FP64
    product with X^T. Both match the oracle and each bound is below the other's primal value."""
    d = synth.make_dataset(600, 150, 6, dtype=dtype, config_id=85)
    sets = synth.node_sets(d.p, d.k, 8, 12, config_id=85)
    with_gram = _problem(d)
    a = with_gram.solve_batch(_specs(with_gram, sets))
    monkeypatch.setenv("CGL_NO_GRAM", "1")
    direct = _problem(d)
    b = direct.solve_batch(_specs(direct, sets))
    for (z0, z1), ra, rb in zip(sets, a, b):
        _check(d, ra, z0, z1)
        _check(d, rb, z0, z1)
        assert rel(ra.primal, rb.primal) <= 2e-6
        assert ra.lower_bound <= rb.primal and rb.lower_bound <= ra.primal


@pytest.mark.parametrize("loss", ["ls", "logistic"])
def test_plain_restart_comparison_matches_oracle(loss, monkeypatch):
    """Alg. 3's restart test without the rounding margin (CGL_RESTART_SLACK=0) restarts far more
    often on the working-precision objective. Every restart takes the residual operand that the
    loss kernel wrote for the restart coefficient (copied into place by the decision kernel), so
    these solves lean on that path: they still match the oracle, and they restart at least as
    often as the same nodes with the default margin."""
    d = synth.make_dataset(500, 300, 6, loss=loss, config_id=91)
    sets = synth.node_sets(d.p, d.k, 10, 15, config_id=91)
    dm = _problem(d)
    a = dm.solve_batch(_specs(dm, sets))
    monkeypatch.setenv("CGL_RESTART_SLACK", "0")
    pl = _problem(d)
    b = pl.solve_batch(_specs(pl, sets))
    for (z0, z1), ra, rb in zip(sets, a, b):
        _check(d, ra, z0, z1)
        _check(d, rb, z0, z1)
    ra_, rb_ = [r.restarts for r in a], [r.restarts for r in b]
    assert sum(rb_) > 0 and sum(rb_) >= sum(ra_), (ra_, rb_)


@pytest.mark.parametrize("loss", ["ls", "logistic"])
def test_operand_reorder_matches_natural_order(loss, monkeypatch):
    """The X pass reads only the prefix of a support-first column order of X~ (re-laid every few
    cycles while the nodes run); with the reordering turned off the same nodes give the same
    certified results within the tolerance, and both match the oracle."""
    d = synth.make_dataset(500, 300, 6, loss=loss, config_id=87)
    sets = synth.node_sets(d.p, d.k, 10, 15, config_id=87)
    re = _problem(d)
    a = re.solve_batch(_specs(re, sets))
    monkeypatch.setenv("CGL_NO_REORDER", "1")
    nat = _problem(d)
    b = nat.solve_batch(_specs(nat, sets))
    for (z0, z1), ra, rb in zip(sets, a, b):
        _check(d, ra, z0, z1)
        assert rel(ra.primal, rb.primal) <= 2e-6
        assert ra.lower_bound <= rb.primal + 1e-12 * abs(rb.primal)
        assert rb.lower_bound <= ra.primal + 1e-12 * abs(ra.primal)


@pytest.mark.parametrize("loss", ["ls", "logistic"])
def test_row_tilings_agree(loss, monkeypatch, tmp_path):
    """The row tilings of the BF16 products (256, 128 and 64 rows per workgroup; the autotuner
    picks one per product shape) give the same certified results within the tolerance, and all
    match the oracle. The BF16 design makes the products' inputs identical in every run; only
    the FP32 summation order differs."""
    monkeypatch.setenv("CGL_TUNE_CACHE", str(tmp_path / "splits.txt"))
    d = synth.make_dataset(700, 300, 6, loss=loss, dtype="bf16", config_id=90)
    sets = synth.node_sets(d.p, d.k, 8, 15, config_id=90)
    out = []
    for tile in ("256", "128", "64"):
        monkeypatch.setenv("CGL_FORCE_TILE", tile)
        prob = _problem(d)
        out.append(prob.solve_batch(_specs(prob, sets)))
        # the tilings in use, as the stats call reports them (code = split-K + 100 * t, with
        # rows = 256 >> t)
        code_x, code_xt = ctx().kernel_stats(14)
        for code in (int(code_x), int(code_xt)):
            assert code % 100 >= 1 and 256 >> (code // 100) == int(tile), (tile, code)
    for (z0, z1), *rs in zip(sets, *out):
        for r in rs:
            _check(d, r, z0, z1)
        for x in rs[1:]:
            ra = rs[0]
            assert rel(ra.primal, x.primal) <= 2e-6
            assert ra.lower_bound <= x.primal + 1e-12 * abs(x.primal)
            assert x.lower_bound <= ra.primal + 1e-12 * abs(ra.primal)


def test_support_prefix_strays_and_overflow(monkeypatch):
    """A support prefix capped far below the union (128 of 300 coordinates) sends every later
    entrant out of the operand as a stray (added to the X-pass product from X~^T) and, past the
    per-slot stray capacity, back into the operand beyond the prefix; the certified results still
    match the oracle."""
    monkeypatch.setenv("CGL_PREFIX_CAP", "128")
    d = synth.make_dataset(500, 300, 6, config_id=88)
    sets = synth.node_sets(d.p, d.k, 6, 15, config_id=88)
    sets.append((np.array([], int), np.array([], int)))
    prob = _problem(d)
    res = prob.solve_batch(_specs(prob, sets))
    for (z0, z1), r in zip(sets, res):
        _check(d, r, z0, z1)


def test_same_inputs_same_bits():
    """Two engines on the same inputs (same context, so the same split-K choice) reproduce each
    other bit for bit, reorders and strays included: no step depends on scheduling."""
    d = synth.make_dataset(500, 300, 6, config_id=89)
    sets = synth.node_sets(d.p, d.k, 12, 15, config_id=89)
    a = _problem(d)
    ra = a.solve_batch(_specs(a, sets))
    b = _problem(d)
    rb = b.solve_batch(_specs(b, sets))
    for x, y in zip(ra, rb):
        assert (x.primal, x.lower_bound, x.iters, x.restarts) == (y.primal, y.lower_bound, y.iters, y.restarts)
        assert np.array_equal(x.beta, y.beta)


def test_caller_output_buffer():
    """solve_batch into a caller's persistent buffer: the same bits as into fresh ones, on two
    calls in a row, the second overwriting the first; wrong buffers are refused. (An engine keeps
    its column order from one call to the next, which moves the rounding, so the comparison is
    between two engines with the same history.)"""
    d = synth.make_dataset(500, 300, 6, config_id=89)
    sets = synth.node_sets(d.p, d.k, 12, 15, config_id=89)
    a = _problem(d)
    prob = _problem(d)
    out = np.full((len(sets), d.p), np.nan)
    for _ in range(2):
        ref = a.solve_batch(_specs(a, sets))
        res = prob.solve_batch(_specs(prob, sets), out=out)
        for i, (x, y) in enumerate(zip(ref, res)):
            assert (x.primal, x.lower_bound, x.iters) == (y.primal, y.lower_bound, y.iters)
            assert np.array_equal(x.beta, out[i]) and np.shares_memory(y.beta, out)
        out[:] = np.nan
    for bad in (np.zeros((len(sets), d.p), dtype=np.float32), np.zeros((len(sets) + 1, d.p)),
                np.zeros((d.p, len(sets))).T):
        with pytest.raises(ValueError):
            prob.solve_batch(_specs(prob, sets), out=bad)


def test_wide_least_squares_mixed():
    """p > n: no Gram matrix; the certificate comes from the FP64 product with X^T."""
    d = synth.make_dataset(120, 300, 5, config_id=86)
    prob = _problem(d)
    sets = synth.node_sets(d.p, d.k, 4, 10, config_id=86)
    res = prob.solve_batch(_specs(prob, sets))
    for (z0, z1), r in zip(sets, res):
        _check(d, r, z0, z1)


def test_config4_subset_full_size():
    """n = 20000, p = 10000, BF16 X: 16 nodes of the benchmark workload are certified to 1e-6;
    the oracle re-evaluates each returned beta to the reported objective and certifies it with
    its own dual point."""
    d = synth.make_config("c4")
    prob = _problem(d)
    sets = synth.node_sets(d.p, d.k, 16, 20, config_id=4)
    res = prob.solve_batch(_specs(prob, sets))
    for (z0, z1), r in zip(sets, res):
        assert r.status == "converged" and r.gap_rel <= 1e-6, r
        ns = oracle.node_sets(d.p, z0, z1)
        P = oracle.primal_value(d.X, d.y, "ls", d.lam2, d.M, d.k, ns, r.beta)
        zeta = -2.0 * (d.X @ r.beta - d.y)
        D = oracle.dual_value(d.X, d.y, "ls", d.lam2, d.M, d.k, ns, zeta)
        assert rel(P, r.primal) <= 1e-10
        assert (P - D) / abs(P) <= 2e-6
        assert r.lower_bound <= P


def test_mixed_warm_start_parent_and_incumbent():
    """Warm starts in the batched engine (the parent's solution, the optimum itself, a random
    vector outside the domain) reach the same certified objective as the cold solve; incumbent
    rules stop a node early with a valid bound."""
    d = synth.make_config("c1")
    prob = _problem(d)
    z0, z1 = [2, 11, 30], [4, 44]
    ref = oracle.solve_node(d.X, d.y, d.loss, d.lam2, d.M, d.k, z0, z1, tol=1e-10)
    parent = oracle.solve_node(d.X, d.y, d.loss, d.lam2, d.M, d.k, [2], [4], tol=1e-10)
    rng = np.random.default_rng(7)
    starts = [ref.beta, parent.beta, 3.0 * rng.standard_normal(d.p)]
    cold = prob.solve_batch(_specs(prob, [(z0, z1)]))[0]
    specs = [prob.node(Z0=z0, Z1=z1, tol=1e-6, max_iter=5000, precision="mixed", warm_start=w)
             for w in starts]
    res = prob.solve_batch(specs)
    for r in res:
        _check(d, r, z0, z1, ref=ref)
        assert abs(r.primal - cold.primal) <= 2e-6 * max(abs(cold.primal), 1.0)
    # from the optimum itself the node certifies in far fewer iterations than cold
    assert res[0].iters < cold.iters
    # incumbent below the bound: pruned; incumbent above the primal: stop and branch
    lo = ref.primal * (1.0 - 1e-3)
    hi = ref.primal * (1.0 + 1e-1)
    rp, rb = prob.solve_batch([
        prob.node(Z0=z0, Z1=z1, tol=1e-9, max_iter=5000, precision="mixed", incumbent=lo),
        prob.node(Z0=z0, Z1=z1, tol=1e-9, max_iter=5000, precision="mixed", incumbent=hi)])
    assert rp.status == "pruned" and lo < rp.lower_bound <= ref.primal
    assert rb.status in ("below_incumbent", "converged") and rb.primal < hi
    assert rb.lower_bound <= ref.primal


@pytest.mark.parametrize("loss", ["poisson", "gamma"])
def test_poisson_gamma_with_given_L_plain_and_mixed(loss):
    """Losses without a global Lipschitz constant take the caller's L; both paths certify the
    nodes to the oracle's objective with the same L. L bounds the curvature within 0.5 of the
    root solution (found first with a cruder bound)."""
    d = synth.make_dataset(400, 60, 3, loss=loss, config_id=91, k_true=3, M=1.0)
    X = d.X * 0.3
    lam = oracle.lambda_max_gram(X)
    crude = 4.0 * lam * math.exp(3.0 * np.abs(X).max()) * (float(np.max(d.y)) if loss == "gamma" else 1.0)
    root = oracle.solve_node(X, d.y, loss, d.lam2, 1.0, d.k, tol=1e-6, L=crude, max_iter=400000)
    u = X @ root.beta
    curv = np.exp(u + 0.5) if loss == "poisson" else d.y * np.exp(-u + 0.5)
    L = 1.2 * float(np.linalg.eigvalsh(X.T @ (curv[:, None] * X))[-1])
    with pytest.raises(_lib.CglError):
        _lib.Problem(ctx(), X, d.y, loss=loss, lam2=d.lam2, M=1.0, k=d.k)  # no L: rejected
    prob = _lib.Problem(ctx(), X, d.y, loss=loss, lam2=d.lam2, M=1.0, k=d.k, L=L)
    sets = synth.node_sets(d.p, d.k, 3, 6, config_id=91)
    for prec in ("f64", "mixed"):
        res = prob.solve_batch([prob.node(Z0=z0, Z1=z1, tol=1e-6, max_iter=100000, precision=prec)
                                for z0, z1 in sets])
        for (z0, z1), r in zip(sets, res):
            ref = oracle.solve_node(X, d.y, loss, d.lam2, 1.0, d.k, z0, z1, tol=1e-9, L=L,
                                    max_iter=400000)
            assert r.status == "converged", (prec, r)
            assert rel(r.primal, ref.primal) <= 1e-6, (prec, r.primal, ref.primal)
            # the relaxation can be exact (box binding on k coordinates): equal up to rounding
            assert r.lower_bound <= ref.primal + 1e-12 * max(1.0, abs(ref.primal))


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_eigen_perspective_on_the_batched_engine(dtype):
    """The eigen-perspective relaxation (App. D.2) on the batched engine, with the shift the
    library proves (cgl_problem_eigen_shift): every node's certified objective matches the
    oracle's eigen-perspective optimum, its bound is the oracle's D_eig at the returned witness and
    never above that optimum, it is at least the perspective bound of the same node, and a server
    gives the same results; shift 0 restores the perspective relaxation on the engine."""
    d = synth.make_dataset(600, 120, 5, loss="ls", dtype=dtype, config_id=81, k_true=5)
    prob = _problem(d)
    sets = [((), ())] + synth.node_sets(d.p, d.k, 6, 10, config_id=81)
    persp = prob.solve_batch(_specs(prob, sets))
    shift = prob.eigen_shift()
    assert 0.0 < shift <= oracle.lambda_min_gram(d.X)
    prob.set_eigen(shift)
    res, duals = prob.solve_batch_dual(_specs(prob, sets))
    for (z0, z1), r, wd, r0 in zip(sets, res, duals, persp):
        ns = oracle.node_sets(d.p, z0, z1)
        ref = oracle.solve_node_eig(d.X, d.y, d.lam2, d.M, d.k, shift, z0, z1, tol=1e-10)
        assert r.status == "converged" and r.gap_rel <= 1e-6, r
        assert rel(r.primal, ref.primal) <= 1e-6, (r.primal, ref.primal)
        assert r.lower_bound <= ref.primal
        Pb = oracle.eig_primal_value(d.X, d.y, d.lam2, d.M, d.k, ns, r.beta, shift)
        assert rel(Pb, r.primal) <= 1e-10, (Pb, r.primal)
        Dw = oracle.eig_dual_value(d.X, d.y, d.lam2, d.M, d.k, ns, wd, shift)
        assert abs(Dw - r.lower_bound) <= 1e-10 * max(abs(r.primal), 1.0), (Dw, r.lower_bound)
        assert r.lower_bound >= r0.lower_bound - 2e-6 * max(abs(r0.primal), 1.0)
    srv = _lib.Server(ctx(), 0, 256)
    tickets = [srv.submit(prob, s) for s in _specs(prob, sets)]
    out = {}
    for _ in range(20000):
        for t, r, _ in srv.poll(64):
            out[t] = r
        if len(out) == len(tickets):
            break
    srv.close()
    for t, r in zip(tickets, res):
        assert out[t].status == "converged"
        assert rel(out[t].primal, r.primal) <= 1e-6
        assert abs(out[t].lower_bound - r.lower_bound) <= 2e-6 * max(abs(r.primal), 1.0)
    prob.set_eigen(0.0)
    back = prob.solve_batch(_specs(prob, sets[:2]))
    for r, r0 in zip(back, persp[:2]):
        assert rel(r.primal, r0.primal) <= 1e-6


def test_split_tuning_persists_across_contexts(tmp_path, monkeypatch):
    """The tilings the autotuner times at engine setup go to the tuning cache file (one line per
    product: arch, pass, rows, k-length, nodes, tiling code = split-K, plus 100 for the 128-row
    tile) and a later context on the same architecture loads them instead of timing again."""
    path = tmp_path / "splits.txt"
    monkeypatch.setenv("CGL_TUNE_CACHE", str(path))
    d = synth.make_dataset(1500, 600, 5, loss="ls", dtype="bf16", config_id=83, k_true=5)
    spec_sets = synth.node_sets(d.p, d.k, 2, 5, config_id=83)
    c1 = _lib.Context(0)
    p1 = _lib.Problem(c1, d.X_store, d.y, loss=d.loss, lam2=d.lam2, M=d.M, k=d.k)
    r1 = p1.solve_batch(_specs(p1, spec_sets))
    lines = path.read_text().splitlines()
    assert len(lines) == 2, lines  # the X pass and the X^T pass each had several candidates
    fields = [ln.split() for ln in lines]
    assert all(len(f) == 6 and f[0].startswith("gfx") and int(f[5]) >= 1 for f in fields)
    assert sorted(int(f[1]) for f in fields) == [0, 1]
    p1.close()
    c1.close()
    c2 = _lib.Context(0)
    p2 = _lib.Problem(c2, d.X_store, d.y, loss=d.loss, lam2=d.lam2, M=d.M, k=d.k)
    r2 = p2.solve_batch(_specs(p2, spec_sets))
    assert path.read_text().splitlines() == lines  # loaded, not timed again
    for a, b in zip(r1, r2):
        assert a.status == b.status == "converged"
        assert rel(a.primal, b.primal) <= 1e-6
    p2.close()
    c2.close()

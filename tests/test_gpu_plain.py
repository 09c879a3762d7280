"""Plain FP64 path on the GPU against the oracle: products, FP64 certificate, full solves."""
import math

import numpy as np
import pytest

import oracle
from paper_2502_09502_amd import _lib, synth

from gpu_util import ctx, rel

pytestmark = pytest.mark.gpu


def _problem(d, L=0.0):
    return _lib.Problem(ctx(), d.X_store, d.y, loss=d.loss, lam2=d.lam2, M=d.M, k=d.k, L=L)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", [(1, 1), (37, 13), (200, 50), (513, 1025), (3000, 700)])
def test_matvec(dtype, shape):
    n, p = shape
    d = synth.make_dataset(max(n, 2), p, 1, dtype=dtype, config_id=70)
    X = d.X[:n] if n < d.n else d.X
    Xs = d.X_store[:n] if n < d.n else d.X_store
    prob = _lib.Problem(ctx(), Xs, np.ones(n), lam2=1e-3, M=2.0, k=1, L=1.0)
    rng = np.random.default_rng(0)
    v = rng.normal(size=p)
    r = rng.normal(size=n)
    np.testing.assert_allclose(prob.matvec(v), X @ v, rtol=1e-12, atol=1e-12 * np.abs(X).sum())
    np.testing.assert_allclose(prob.matvec(r, trans=True), X.T @ r, rtol=1e-12,
                               atol=1e-12 * np.abs(X).sum())


def test_lipschitz_power_iteration():
    d = synth.make_config("c1")
    prob = _problem(d)
    ref = oracle.lipschitz(d.X, "ls")
    assert ref <= prob.L <= ref * 1.0025


@pytest.mark.parametrize("loss", ["ls", "logistic", "sqhinge"])
def test_certify_matches_oracle(loss):
    d = synth.make_dataset(300, 90, 5, loss=loss, config_id=71)
    prob = _problem(d)
    rng = np.random.default_rng(3)
    for trial in range(4):
        perm = rng.permutation(d.p)
        z0, z1 = perm[:trial * 3], perm[trial * 3:trial * 3 + trial]
        ns = oracle.node_sets(d.p, z0, z1)
        beta = oracle.prox_node(rng.normal(size=d.p), 50.0, d.M, d.k, ns)
        P, D = prob.certify(beta, z0, z1)
        Pref = oracle.primal_value(d.X, d.y, loss, d.lam2, d.M, d.k, ns, beta)
        zeta = -oracle.get_loss(loss).grad(d.X @ beta, d.y)
        Dref = oracle.dual_value(d.X, d.y, loss, d.lam2, d.M, d.k, ns, zeta)
        assert rel(P, Pref) <= 1e-11 and rel(D, Dref) <= 1e-11


def _compare(d, res, ref, ns, tol=1e-6):
    assert res.status == "converged", res
    assert res.gap_rel <= tol
    assert rel(res.primal, ref.primal) <= 1e-6, (res.primal, ref.primal)
    assert res.lower_bound <= ref.primal  # never above the oracle's certified optimum
    # the returned beta evaluates (in the oracle) to the reported objective
    Pb = oracle.primal_value(d.X, d.y, d.loss, d.lam2, d.M, d.k, ns, res.beta)
    assert rel(Pb, res.primal) <= 1e-10


@pytest.mark.parametrize("loss", ["ls", "logistic", "sqhinge"])
def test_config1_root(loss):
    d = synth.make_config("c1") if loss == "ls" else synth.make_dataset(
        200, 50, 5, loss=loss, config_id=1)
    ref = oracle.solve_node(d.X, d.y, loss, d.lam2, d.M, d.k, tol=1e-9)
    res = _problem(d).solve(tol=1e-6)
    _compare(d, res, ref, oracle.node_sets(d.p))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("seed", range(3))
def test_small_nodes(dtype, seed):
    d = synth.make_dataset(700, 300, 10, loss=["ls", "logistic"][seed % 2], dtype=dtype,
                           config_id=72 + seed)
    prob = _problem(d)
    sets = synth.node_sets(d.p, d.k, 3, 20, config_id=72 + seed)
    for z0, z1 in sets:
        ns = oracle.node_sets(d.p, z0, z1)
        ref = oracle.solve_node(d.X, d.y, d.loss, d.lam2, d.M, d.k, z0, z1, tol=1e-9)
        res = prob.solve(z0, z1, tol=1e-6)
        _compare(d, res, ref, ns)


def test_edge_cases():
    d = synth.make_dataset(120, 40, 4, config_id=75)
    prob = _problem(d)
    # infeasible node
    r = prob.solve(Z1=[0, 1, 2, 3, 4])
    assert r.status == "infeasible" and r.lower_bound == math.inf
    # every coordinate fixed to zero: beta = 0, P = D = f(0)
    r = prob.solve(Z0=np.arange(40))
    f0 = float(d.y @ d.y)
    assert r.status == "converged" and rel(r.primal, f0) < 1e-14 and np.all(r.beta == 0)
    # k' = 0 with free coordinates
    r = prob.solve(Z1=[3, 5, 7, 9])
    ref = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, d.k, (), [3, 5, 7, 9], tol=1e-9)
    assert rel(r.primal, ref.primal) <= 1e-6 and r.lower_bound <= ref.primal
    # iteration cap: still a valid bound
    r = prob.solve(max_iter=3)
    ref = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, d.k, tol=1e-10)
    assert r.status == "not_converged" and r.iters == 3 and r.lower_bound <= ref.primal
    # invalid arguments raise
    with pytest.raises(_lib.CglError):
        prob.solve(Z0=[1], Z1=[1])
    with pytest.raises(_lib.CglError):
        prob.solve(Z0=[40])
    # warm start from the oracle optimum converges at once
    r = prob.solve(warm_start=ref.beta, tol=1e-6)
    assert r.status == "converged" and r.iters <= 20


def test_config2_full_size_properties():
    """n = 10000, p = 5000 FP64 and FP32: the solve certifies 1e-6, the oracle evaluates the
    returned beta to the same objective, and certifies it optimal by its own dual."""
    for name in ("c2_f64", "c2_f32"):
        d = synth.make_config(name)
        prob = _problem(d)
        res = prob.solve(tol=1e-6)
        assert res.status == "converged" and res.gap_rel <= 1e-6
        ns = oracle.node_sets(d.p)
        P = oracle.primal_value(d.X, d.y, "ls", d.lam2, d.M, d.k, ns, res.beta)
        zeta = -2.0 * (d.X @ res.beta - d.y)
        D = oracle.dual_value(d.X, d.y, "ls", d.lam2, d.M, d.k, ns, zeta)
        assert rel(P, res.primal) <= 1e-10
        assert (P - D) / abs(P) <= 2e-6
        assert res.lower_bound <= P
        Pc, Dc = prob.certify(res.beta)
        assert rel(Pc, P) <= 1e-11 and rel(Dc, D) <= 1e-10


def test_eigen_perspective_relaxation():
    """Eigen-perspective relaxation (App. D.2) on the FP64 path: the certified objective matches
    the oracle's, the bound is at least the perspective one and never above the oracle's optimum;
    other losses, negative shifts and cgl_certify reject it."""
    d = synth.make_dataset(300, 60, 5, loss="ls", config_id=77, k_true=5)
    lmin = oracle.lambda_min_gram(d.X)
    assert lmin > 0
    shift = lmin * (1.0 - 1e-6)
    prob = _problem(d)
    sets = [((), ()), ([3, 11], [7]), ([], [1, 2])]
    std = [prob.solve(Z0=z0, Z1=z1, tol=1e-7) for z0, z1 in sets]
    prob.set_eigen(shift)
    for (z0, z1), s0 in zip(sets, std):
        r = prob.solve(Z0=z0, Z1=z1, tol=1e-7)
        ref = oracle.solve_node_eig(d.X, d.y, d.lam2, d.M, d.k, shift, z0, z1, tol=1e-10)
        assert r.status == "converged", r
        assert rel(r.primal, ref.primal) <= 1e-6, (r.primal, ref.primal)
        assert r.lower_bound <= ref.primal
        assert r.lower_bound >= s0.lower_bound - 1e-6 * abs(s0.primal)
    with pytest.raises(_lib.CglError):
        prob.certify(np.zeros(d.p))
    with pytest.raises(_lib.CglError):
        prob.set_eigen(-1.0)
    prob.set_eigen(0.0)  # back to the perspective relaxation
    r = prob.solve(tol=1e-7)
    assert rel(r.primal, std[0].primal) <= 1e-6
    dl = synth.make_dataset(300, 60, 5, loss="logistic", config_id=77)
    with pytest.raises(_lib.CglError):
        _problem(dl).set_eigen(0.1)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_non_finite_device_X_rejected(dtype):
    """A design given in device memory is checked for NaN and infinity on the device."""
    from paper_2502_09502_amd.devmem import DeviceArray

    d = synth.make_dataset(64, 24, 3, dtype=dtype, config_id=93)
    Xd = DeviceArray.from_numpy(d.X_store)
    ok = _lib.Problem(ctx(), Xd, d.y, loss="ls", lam2=d.lam2, M=d.M, k=d.k)
    assert ok.L > 0
    ok.close()
    # bit patterns of NaN and +infinity in the stored type (BF16: exponent all ones)
    bads = {"f64": (np.nan, np.inf), "f32": (np.float32(np.nan), np.float32(np.inf)),
            "bf16": (np.uint16(0x7FC0), np.uint16(0x7F80))}[dtype]
    for bad in bads:
        Xh = d.X_store.copy()
        Xh[5, 7] = bad
        Xb = DeviceArray.from_numpy(Xh)
        with pytest.raises(_lib.CglError) as e:
            _lib.Problem(ctx(), Xb, d.y, loss="ls", lam2=d.lam2, M=d.M, k=d.k)
        assert e.value.code == _lib.E_INVAL and "non-finite" in str(e.value)
        Xb.free()
    Xd.free()


@pytest.mark.parametrize("n,p,dtype", [(300, 60, "f64"), (2000, 1000, "f32"), (1500, 777, "bf16")])
def test_eigen_shift_is_certified(n, p, dtype):
    """The library proves an eigen-perspective shift before it accepts it (App. D.2 needs
    shift <= lambda_min(X^T X)): the largest shift its FP64 Cholesky test proves lies just below
    the exact lambda_min of the stored design (a dense eigen-solver on the CPU), a shift above
    lambda_min is refused, and a design with n < p accepts only 0."""
    d = synth.make_dataset(n, p, 5, loss="ls", dtype=dtype, config_id=78, k_true=5)
    lmin = oracle.lambda_min_gram(d.X)
    prob = _problem(d)
    auto = prob.eigen_shift()
    assert lmin * (1.0 - 1e-5) <= auto <= lmin, (auto, lmin)
    prob.set_eigen(auto)
    prob.set_eigen(lmin * (1.0 - 1e-4))
    with pytest.raises(_lib.CglError) as e:
        prob.set_eigen(lmin * (1.0 + 1e-4))
    assert e.value.code == _lib.E_INVAL and "not certified" in str(e.value)
    prob.set_eigen(0.0)
    wide = synth.make_dataset(40, 60, 5, loss="ls", config_id=79, k_true=5)
    pw = _problem(wide)
    assert pw.eigen_shift() == 0.0
    with pytest.raises(_lib.CglError):
        pw.set_eigen(1e-3)

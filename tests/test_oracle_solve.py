"""Pins of the oracle's losses, conjugates, dual bound and restarted-FISTA solve against closed
forms (ridge, bounded least squares), brute-force enumeration of supports, the l1 relaxation of
App. C.2, the Fenchel-Young equality of the loss conjugates (App. D.1) and finite differences."""
import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear, minimize, minimize_scalar

import oracle
from paper_2502_09502_amd import synth


def _tiny(n=20, p=8, loss="ls", seed=0):
    return synth.make_dataset(n, p, 2, loss=loss, config_id=50 + seed, k_true=2)


# ------------------------------------------------------------------------------- losses


def _responses(loss, rng, n):
    if loss == "ls":
        return rng.normal(size=n)
    if loss == "poisson":
        return rng.poisson(2.0, size=n).astype(float)
    if loss == "gamma":
        return rng.gamma(2.0, 1.0, size=n)
    return rng.choice([-1.0, 1.0], size=n)


ALL_LOSSES = ["ls", "logistic", "sqhinge", "poisson", "gamma"]


@pytest.mark.parametrize("loss", ALL_LOSSES)
def test_loss_gradient_finite_difference(loss):
    rng = np.random.default_rng(1)
    y = _responses(loss, rng, 7)
    L = oracle.get_loss(loss)
    u = rng.normal(size=7)
    g = L.grad(u, y)
    for i in range(7):
        e = np.zeros(7)
        e[i] = 1e-6
        fd = (L.f(u + e, y) - L.f(u - e, y)) / 2e-6
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("loss", ALL_LOSSES)
def test_loss_conjugate_fenchel_young_and_sup(loss):
    """F(u) + F*(s) = s^T u at s = grad F(u); F*(s) = sup_u s^T u - F(u) (coordinatewise)."""
    rng = np.random.default_rng(2)
    n = 6
    y = _responses(loss, rng, n)
    L = oracle.get_loss(loss)
    u = rng.normal(size=n)
    s = L.grad(u, y)
    # conj_neg(zeta) = F*(-zeta): evaluate F*(s) with zeta = -s
    assert L.f(u, y) + L.conj_neg(-s, y) == pytest.approx(float(s @ u), rel=1e-12, abs=1e-12)
    # sup over u of s^T u - F(u), one coordinate at a time (F is separable)
    total = 0.0
    for i in range(n):
        yi = y[i:i + 1]
        fn = lambda t: -(s[i] * t - L.f(np.array([t]), yi))
        res = minimize_scalar(fn, bounds=(-60, 60), method="bounded", options={"xatol": 1e-12})
        total += -res.fun
    assert L.conj_neg(-s, y) == pytest.approx(total, rel=1e-7, abs=1e-9)


def test_logistic_conjugate_domain():
    y = np.array([1.0, -1.0])
    assert oracle.Logistic.conj_neg(np.array([0.5, 0.5]), y) == math.inf  # q_2 = -0.5
    assert oracle.Logistic.conj_neg(np.array([1.0, -1.0]), y) == 0.0  # q = 1: 1 log 1 + 0 log 0


# ------------------------------------------------------------------------------- dual bound


@pytest.mark.parametrize("loss", ALL_LOSSES)
def test_weak_duality_random_points(loss):
    d = _tiny(loss=loss)
    ns = oracle.node_sets(d.p, Z0=[1], Z1=[4])
    rng = np.random.default_rng(3)
    for _ in range(20):
        beta = oracle.prox_node(rng.normal(size=d.p), 5.0, d.M, d.k, ns)
        P = oracle.primal_value(d.X, d.y, loss, d.lam2, d.M, d.k, ns, beta)
        if loss == "ls":
            zeta = rng.normal(size=d.n) * 2
        elif loss == "logistic":
            zeta = d.y * rng.uniform(0, 1, size=d.n)
        elif loss == "sqhinge":  # -y zeta <= 0
            zeta = d.y * rng.uniform(0, 3, size=d.n)
        elif loss == "poisson":  # y - zeta >= 0
            zeta = d.y - rng.uniform(0, 2, size=d.n)
        else:  # gamma: (1 + zeta) / y >= 0
            zeta = -1.0 + rng.uniform(0, 3, size=d.n)
        D = oracle.dual_value(d.X, d.y, loss, d.lam2, d.M, d.k, ns, zeta)
        assert D <= P + 1e-9


# ------------------------------------------------------------------------------- the solve


def test_ridge_closed_form_when_budget_covers_free_set():
    """k' >= |F| and M not binding: P_conv is ridge regression on the non-zero-fixed columns."""
    d = synth.make_dataset(40, 8, 8, loss="ls", config_id=61, k_true=2, M=100.0)
    Z0 = [2, 5]
    S = [j for j in range(8) if j not in Z0]
    XS = d.X[:, S]
    b = np.linalg.solve(XS.T @ XS + d.lam2 * np.eye(len(S)), XS.T @ d.y)
    ref = float(np.sum((XS @ b - d.y) ** 2) + d.lam2 * b @ b)
    r = oracle.solve_node(d.X, d.y, "ls", d.lam2, 100.0, 8, Z0=Z0, tol=1e-10)
    assert r.status == oracle.CONVERGED
    assert r.primal == pytest.approx(ref, rel=1e-9)
    assert r.lower_bound <= ref * (1 + 1e-12)
    np.testing.assert_allclose(r.beta[S], b, atol=1e-5)


def test_bounded_least_squares_when_box_binds():
    d = synth.make_dataset(40, 6, 6, loss="ls", config_id=62, k_true=3)
    M = 0.4
    A = np.vstack([d.X, math.sqrt(d.lam2) * np.eye(6)])
    rhs = np.concatenate([d.y, np.zeros(6)])
    res = lsq_linear(A, rhs, bounds=(-M, M), tol=1e-14, method="bvls")
    ref = float(np.sum((A @ res.x - rhs) ** 2))
    r = oracle.solve_node(d.X, d.y, "ls", d.lam2, M, 6, tol=1e-10)
    assert r.primal == pytest.approx(ref, rel=1e-9)
    assert np.max(np.abs(r.beta)) <= M * (1 + 1e-12)
    assert np.any(np.abs(res.x) >= M * (1 - 1e-9))  # the box does bind


def test_fixed_in_support_equals_box_ridge_on_support():
    """Z1 = S, Z0 = the rest, k = |S|: the node is the box ridge problem on S, i.e. P_MIP there."""
    d = _tiny(p=8, seed=3)
    S = [1, 6]
    Z0 = [j for j in range(8) if j not in S]
    A = np.vstack([d.X[:, S], math.sqrt(d.lam2) * np.eye(2)])
    rhs = np.concatenate([d.y, np.zeros(2)])
    res = lsq_linear(A, rhs, bounds=(-d.M, d.M), tol=1e-14, method="bvls")
    ref = float(np.sum((A @ res.x - rhs) ** 2))
    r = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, 2, Z0=Z0, Z1=S, tol=1e-10)
    assert r.primal == pytest.approx(ref, rel=1e-9)
    assert oracle.brute_force_mip(d.X, d.y, "ls", d.lam2, d.M, 2, Z0=Z0, Z1=S) == pytest.approx(
        ref, rel=1e-9)


def test_all_fixed_to_zero_gives_f0():
    d = _tiny()
    r = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, d.k, Z0=list(range(d.p)), tol=1e-12)
    f0 = float(d.y @ d.y)
    assert r.primal == f0 and r.lower_bound == pytest.approx(f0, rel=1e-15)
    assert np.all(r.beta == 0)


def test_infeasible_node():
    d = _tiny()
    r = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, 2, Z1=[0, 1, 2])
    assert r.status == oracle.INFEASIBLE and r.lower_bound == math.inf


def _l1_relaxation(X, y, loss, lam2, M, k, Z0=()):
    """App. C.2: min f(X b) + lambda2 ||b||^2 s.t. ||b||_1 <= k M, ||b||_inf <= M (b_Z0 = 0), as a
    smooth problem in b = b+ - b-, solved by SLSQP."""
    p = X.shape[1]
    L = oracle.get_loss(loss)
    keep = np.array([j not in set(Z0) for j in range(p)])

    def obj(v):
        b = (v[:p] - v[p:]) * keep
        return L.f(X @ b, y) + lam2 * b @ b

    cons = [{"type": "ineq", "fun": lambda v: k * M - np.sum(v)}]
    res = minimize(obj, np.full(2 * p, 1e-3), method="SLSQP", bounds=[(0, M)] * (2 * p),
                   constraints=cons, options={"ftol": 1e-14, "maxiter": 2000})
    return float(res.fun)


@pytest.mark.parametrize("loss", ["ls", "logistic", "sqhinge"])
@pytest.mark.parametrize("seed", range(4))
def test_bound_sandwich_brute_force(loss, seed):
    """P_l1 <= P_conv ~ D <= P_MIP: the certified bound is valid (never above the exact k-sparse
    optimum found by enumeration) and tight (not below the looser l1 relaxation)."""
    d = _tiny(n=25, p=8, loss=loss, seed=seed)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(d.p)
    Z0 = [int(perm[0])] if seed % 2 else []
    Z1 = [int(perm[1])] if seed >= 2 else []
    k = 2
    r = oracle.solve_node(d.X, d.y, loss, d.lam2, d.M, k, Z0=Z0, Z1=Z1, tol=1e-9)
    assert r.status == oracle.CONVERGED
    pmip = oracle.brute_force_mip(d.X, d.y, loss, d.lam2, d.M, k, Z0=Z0, Z1=Z1)
    assert r.lower_bound <= pmip
    assert r.primal <= pmip * (1 + 1e-9)
    if not Z1:
        pl1 = _l1_relaxation(d.X, d.y, loss, d.lam2, d.M, k, Z0=Z0)
        assert pl1 <= r.primal * (1 + 1e-7)
        assert r.lower_bound >= pl1 - 1e-6 * max(1.0, abs(pl1))


def test_gap_closes_and_beta_is_feasible_on_config1():
    d = synth.make_config("c1")
    r = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, d.k, tol=1e-8)
    assert r.status == oracle.CONVERGED and r.gap_rel <= 1e-8
    assert oracle.in_dom_g(r.beta, d.k, d.M, slack=1e-12)
    # D is below the objective of a feasible k-sparse point (box ridge on the top-k support)
    S = np.argsort(-np.abs(r.beta))[: d.k]
    A = np.vstack([d.X[:, S], math.sqrt(d.lam2) * np.eye(d.k)])
    res = lsq_linear(A, np.concatenate([d.y, np.zeros(d.k)]), bounds=(-d.M, d.M), tol=1e-14)
    feas = float(np.sum((A @ res.x - np.concatenate([d.y, np.zeros(d.k)])) ** 2))
    assert r.lower_bound <= feas


def test_restart_beats_plain_fista_and_pgd():
    """Qualitative claim of Sec. 4.2: value restart needs fewer iterations than FISTA and PGD."""
    d = synth.make_config("c1")
    args = (d.X, d.y, "ls", d.lam2, d.M, d.k)
    r = oracle.solve_node(*args, tol=1e-6)
    f = oracle.solve_node(*args, tol=1e-6, restart=False)
    g = oracle.solve_node(*args, tol=1e-6, momentum=False)
    assert r.iters < f.iters and r.iters < g.iters
    assert abs(r.primal - f.primal) <= 2e-6 * r.primal


def test_lipschitz_matches_eigenvalue_and_lanczos_path():
    rng = np.random.default_rng(9)
    X = rng.normal(size=(300, 2100))
    lam = float(np.linalg.eigvalsh(X.T @ X)[-1])  # dense reference
    assert oracle.lambda_max_gram(X) == pytest.approx(lam, rel=1e-10)  # Lanczos branch (p > 2000)
    assert oracle.lipschitz(X, "ls") == pytest.approx(2 * lam, rel=1e-10)
    assert oracle.lipschitz(X, "logistic") == pytest.approx(lam / 4, rel=1e-10)
    assert oracle.lipschitz(X, "sqhinge") == pytest.approx(2 * lam, rel=1e-10)


def test_budget_exhausted_by_fixed_in_set():
    """k' = k - |Z1| = 0: g restricted to the free set is the indicator of beta_F = 0, so the node
    is the box ridge problem on Z1 alone (closed form by bounded least squares)."""
    d = synth.make_dataset(150, 40, 4, config_id=82)
    Z1 = [3, 5, 7, 9]
    r = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, 4, (), Z1, tol=1e-10)
    A = np.vstack([d.X[:, Z1], math.sqrt(d.lam2) * np.eye(4)])
    rhs = np.concatenate([d.y, np.zeros(4)])
    res = lsq_linear(A, rhs, bounds=(-d.M, d.M), tol=1e-14, method="bvls")
    ref = float(np.sum((A @ res.x - rhs) ** 2))
    assert r.status == oracle.CONVERGED and r.iters < 1000
    assert r.primal == pytest.approx(ref, rel=1e-9)
    free = [j for j in range(40) if j not in Z1]
    assert np.all(r.beta[free] == 0.0)


def test_squared_hinge_conjugate_closed_form_and_domain():
    """One coordinate by hand (y = 1): f(u) = (1 - u)^2 for u < 1; at u = 0.5 the slope is
    s = -1 and F*(s) = sup_t s t - f(t) is attained at t = 1 + s/2 = 0.5: -0.5 - 0.25 = -0.75,
    which is h(-y zeta) = h(s) = s + s^2/4 with zeta = -s. Outside the domain (-y zeta > 0) the
    conjugate is infinite."""
    y = np.array([1.0])
    assert oracle.SquaredHinge.conj_neg(np.array([1.0]), y) == pytest.approx(-0.75, abs=1e-15)
    assert oracle.SquaredHinge.conj_neg(np.array([-0.5]), y) == math.inf
    assert oracle.SquaredHinge.f(np.array([2.0]), y) == 0.0  # margin met: no loss


@pytest.mark.parametrize("loss", ["poisson", "gamma"])
def test_poisson_gamma_node_solve_with_given_L(loss):
    """Losses without a global Lipschitz constant: with an L that bounds the curvature along the
    path, Alg. 3 certifies the node, and the bound is below the brute-force k-sparse optimum."""
    d = synth.make_dataset(60, 8, 2, loss=loss, config_id=90, k_true=2, M=1.0)
    X, y = d.X * 0.5, d.y  # milder curvature
    lam = oracle.lambda_max_gram(X)
    L = 8.0 * lam * (math.exp(2.0 * np.abs(X).max()) if loss == "poisson" else
                     float(np.max(y)) * math.exp(2.0 * np.abs(X).max()))
    with pytest.raises(ValueError):
        oracle.lipschitz(X, loss)
    r = oracle.solve_node(X, y, loss, d.lam2, 1.0, 2, Z0=[1], tol=1e-8, L=L, max_iter=200000)
    assert r.status == oracle.CONVERGED
    pmip = oracle.brute_force_mip(X, y, loss, d.lam2, 1.0, 2, Z0=[1])
    # the relaxation can be exact here (the box binds on k coordinates): equality up to rounding
    slack = max(1.0, abs(pmip))
    assert r.lower_bound <= pmip + 1e-13 * slack and r.primal <= pmip + 1e-9 * slack


# ------------------------------------------------------------------ eigen-perspective relaxation


def _eig_data(seed=0, n=40, p=8):
    d = synth.make_dataset(n, p, 2, loss="ls", config_id=95 + seed, k_true=2)
    return d, oracle.lambda_min_gram(d.X)


def test_lambda_min_matches_dense_eigenvalues():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(60, 12))
    assert oracle.lambda_min_gram(X) == pytest.approx(float(np.linalg.eigvalsh(X.T @ X)[0]),
                                                      rel=1e-12)


def test_eig_with_zero_shift_is_the_perspective_relaxation():
    d, _ = _eig_data(0)
    r0 = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, 2, Z0=[3], tol=1e-10)
    r1 = oracle.solve_node_eig(d.X, d.y, d.lam2, d.M, 2, 0.0, Z0=[3], tol=1e-10)
    assert r1.status == oracle.CONVERGED
    assert r1.primal == pytest.approx(r0.primal, rel=1e-9)
    assert r1.lower_bound == pytest.approx(r0.lower_bound, rel=1e-8)


def test_eig_ridge_closed_form_when_budget_covers_free_set():
    """All z_j = 1: the eigen-perspective problem is ridge regression with lambda2 for any
    admissible shift (s ||b||^2 - s ||b||^2 cancels)."""
    d = synth.make_dataset(40, 6, 6, loss="ls", config_id=97, k_true=2, M=100.0)
    s = 0.9 * oracle.lambda_min_gram(d.X)
    b = np.linalg.solve(d.X.T @ d.X + d.lam2 * np.eye(6), d.X.T @ d.y)
    ref = float(np.sum((d.X @ b - d.y) ** 2) + d.lam2 * b @ b)
    r = oracle.solve_node_eig(d.X, d.y, d.lam2, 100.0, 6, s, tol=1e-11)
    assert r.primal == pytest.approx(ref, rel=1e-9)
    assert r.lower_bound <= ref * (1 + 1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_eig_bound_valid_and_tighter(seed):
    """perspective bound <= eigen-perspective bound <= P_MIP (brute force)."""
    d, lmin = _eig_data(seed)
    assert lmin > 0
    rng = np.random.default_rng(seed)
    perm = rng.permutation(d.p)
    Z0 = [int(perm[0])] if seed % 2 else []
    Z1 = [int(perm[1])] if seed >= 2 else []
    k = 2
    std = oracle.solve_node(d.X, d.y, "ls", d.lam2, d.M, k, Z0=Z0, Z1=Z1, tol=1e-10)
    eig = oracle.solve_node_eig(d.X, d.y, d.lam2, d.M, k, lmin, Z0=Z0, Z1=Z1, tol=1e-10)
    assert eig.status == oracle.CONVERGED
    pmip = oracle.brute_force_mip(d.X, d.y, "ls", d.lam2, d.M, k, Z0=Z0, Z1=Z1)
    assert eig.lower_bound <= pmip * (1 + 1e-12)
    assert eig.lower_bound >= std.lower_bound - 1e-8 * abs(std.primal)


def test_eig_dual_is_weak_duality():
    """D_eig(b_hat) <= the eigen-perspective objective at any point, for any b_hat."""
    d, lmin = _eig_data(1)
    ns = oracle.node_sets(d.p, [2], [5])
    rng = np.random.default_rng(5)
    for _ in range(20):
        bh = rng.normal(size=d.p)
        D = oracle.eig_dual_value(d.X, d.y, d.lam2, d.M, 2, ns, bh, lmin)
        b = oracle.prox_node(rng.normal(size=d.p), 3.0, d.M, 2, ns)
        P = oracle.eig_primal_value(d.X, d.y, d.lam2, d.M, 2, ns, b, lmin)
        assert D <= P + 1e-9

"""Pins of the oracle's prox of g* (Alg. 1), prox of g (Moreau identity), g (Alg. 2) and g* (Lemma 2)
against things other than the oracle itself: a generic nested 1-D convex solve, the KKT system of
eq. (10), a Lagrangian water-filling of eq. (7), a linear program for Lemma 2, textbook special
cases, the Fenchel-Young equality and hand-derived worked examples."""
import math
import os

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "prox_g_worked_examples.txt")
PHI = (math.sqrt(5.0) - 1.0) / 2.0


def _golden_min(fn, lo, hi, iters=160):
    """Golden-section minimisation of a 1-D convex function on [lo, hi]."""
    a, b = lo, hi
    c = b - PHI * (b - a)
    d = a + PHI * (b - a)
    fc, fd = fn(c), fn(d)
    for _ in range(iters):
        if fc <= fd:
            b, d, fd = d, c, fc
            c = b - PHI * (b - a)
            fc = fn(c)
        else:
            a, c, fc = c, d, fd
            d = a + PHI * (b - a)
            fd = fn(d)
    return 0.5 * (a + b)


def _huber_scalar(a, M):
    a = abs(a)
    return 0.5 * a * a if a <= M else M * a - 0.5 * M * M


def generic_prox_gstar(mu, rho, M, k):
    """argmin 1/2||alpha - mu||^2 + rho TopSum_k(H_M(alpha)), using
    TopSum_k(h) = min_t k t + sum (h_j - t)_+ : for fixed t the problem splits into 1-D convex
    problems (golden section on [min(0, mu_j), max(0, mu_j)]); the outer problem is convex in t
    (golden section on [0, max H_M(mu)])."""
    mu = np.asarray(mu, float)

    def inner(t):
        alphas, total = [], rho * k * t
        for m in mu:
            fn = lambda a: 0.5 * (a - m) ** 2 + rho * max(_huber_scalar(a, M) - t, 0.0)
            a = _golden_min(fn, min(0.0, m), max(0.0, m), iters=120)
            alphas.append(a)
            total += fn(a)
        return total, np.asarray(alphas)

    hmax = max(_huber_scalar(m, M) for m in mu)
    t_star = _golden_min(lambda t: inner(t)[0], 0.0, hmax + 1e-12, iters=120)
    return inner(t_star)[1]


def kkt_residual(mu, alpha, rho, M, k):
    """Optimality of alpha for eq. (10): mu_j - alpha_j = rho w_j clip(alpha_j, -M, M) with
    w in [0, 1]^p, sum w = k (when more than k entries have H_M > 0), w_j = 1 above the k-th largest
    H_M(alpha), w_j = 0 below it. Returns the largest violation."""
    h = oracle.huber(alpha, M)
    hs = np.sort(h)[::-1]
    kth = hs[k - 1] if k <= len(h) else 0.0
    clip = np.clip(alpha, -M, M)
    viol = 0.0
    wsum = 0.0
    free = []
    scale = max(1.0, np.max(np.abs(mu)))
    for j in range(len(mu)):
        r = mu[j] - alpha[j]
        tie = abs(h[j] - kth) <= 1e-9 * max(1.0, kth)
        if abs(clip[j]) < 1e-14:
            viol = max(viol, abs(r) / scale)
            continue
        w = r / (rho * clip[j])
        if tie and kth > 0:
            viol = max(viol, max(0.0, -w), max(0.0, w - 1.0))
            free.append(w)
            wsum += w
        elif h[j] > kth:
            viol = max(viol, abs(w - 1.0))
            wsum += 1.0
        else:
            viol = max(viol, abs(w))
    if k <= len(h) and kth > 0:
        viol = max(viol, abs(wsum - k) / k)
    return viol


def _cases(seed, count):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        p = int(rng.integers(1, 8))
        k = int(rng.integers(1, p + 2))
        M = float(rng.choice([0.3, 1.0, 2.0, 50.0]))
        rho = float(rng.choice([0.2, 1.0, 3.0]))
        mu = rng.normal(0, 2.0, size=p) * float(rng.choice([0.5, 1.0, 4.0]))
        yield mu, rho, M, k


@pytest.mark.parametrize("case", list(_cases(0, 40)))
def test_prox_gstar_matches_generic_solve(case):
    mu, rho, M, k = case
    got = oracle.prox_gstar(mu, rho, M, k)
    ref = generic_prox_gstar(mu, rho, M, k)
    assert np.max(np.abs(got - ref)) <= 1e-7 * max(1.0, np.max(np.abs(mu)))


@pytest.mark.parametrize("case", list(_cases(1, 60)))
def test_prox_gstar_kkt(case):
    mu, rho, M, k = case
    alpha = oracle.prox_gstar(mu, rho, M, k)
    assert kkt_residual(mu, alpha, rho, M, k) <= 1e-9


def test_prox_gstar_kkt_with_ties_and_zeros():
    mu = np.array([3.0, -3.0, 3.0, 0.0, 1.0, -0.5, 0.0])
    for k in (1, 2, 3, 5):
        for M in (0.5, 2.0, 10.0):
            alpha = oracle.prox_gstar(mu, 1.5, M, k)
            assert kkt_residual(mu, alpha, 1.5, M, k) <= 1e-9
            assert alpha[3] == 0.0 and alpha[6] == 0.0


def test_special_case_k_ge_p_is_elementwise_huber_prox():
    """k >= p: g* = sum H_M, whose prox is the elementwise Huber prox (Beck 2017, Ex. 6.54):
    a/(1+rho) if |a| <= M(1+rho), else a - rho M sgn(a)."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        p = int(rng.integers(1, 30))
        mu = rng.normal(0, 3, size=p)
        rho, M = float(rng.uniform(0.1, 3)), float(rng.uniform(0.2, 4))
        ref = np.where(np.abs(mu) <= M * (1 + rho), mu / (1 + rho), mu - rho * M * np.sign(mu))
        np.testing.assert_allclose(oracle.prox_gstar(mu, rho, M, p), ref, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(oracle.prox_gstar(mu, rho, M, p + 3), ref, rtol=1e-13, atol=1e-13)


def test_special_case_k_zero_is_identity():
    mu = np.array([1.0, -2.0, 0.5])
    np.testing.assert_array_equal(oracle.prox_gstar(mu, 2.0, 1.0, 0), mu)


def test_special_case_large_M_is_topk_shrink():
    """M -> inf: g* = 1/2 TopSum_k(alpha^2) (k-support norm setting, Sec. 3.3). With one element far
    above the rest and k = 1 the top entry is shrunk by 1/(1+rho) and the rest are unchanged."""
    mu = np.array([100.0, 1.0, -0.5])
    alpha = oracle.prox_gstar(mu, 1.0, 1e9, 1)
    np.testing.assert_allclose(alpha, [50.0, 1.0, -0.5], rtol=1e-14)


def _read_golden():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split("|")
            parts = lhs.split()
            kind, rho, M, k = parts[0], float(parts[1]), float(parts[2]), int(parts[3])
            x = np.array([float(v) for v in parts[4:]])
            expected = np.array([float(v) for v in rhs.split()])
            rows.append((kind, rho, M, k, x, expected))
    return rows


@pytest.mark.parametrize("row", _read_golden())
def test_worked_examples(row):
    kind, rho, M, k, x, expected = row
    for sign in (1.0, -1.0):  # a sign flip of the input flips alpha and beta (Lemma 3)
        xs = sign * x
        if kind == "prox_gstar":
            np.testing.assert_allclose(oracle.prox_gstar(xs, rho, M, k), sign * expected,
                                       rtol=1e-14, atol=1e-14)
        elif kind == "prox_g":
            np.testing.assert_allclose(oracle.prox_g(xs, rho, M, k), sign * expected,
                                       rtol=1e-14, atol=1e-14)
        elif kind == "g_value":
            assert oracle.g_value(xs, k, M) == pytest.approx(expected[0], rel=1e-14)
        elif kind == "gstar":
            assert oracle.gstar_value(xs, k, M) == pytest.approx(expected[0], rel=1e-14)


# ---------------------------------------------------------------- g (Alg. 2) and g* (Lemma 2)


def g_waterfill(beta, k, M):
    """g(beta) of eq. (7) from its Lagrangian: z_j = clip(|beta_j| / tau, |beta_j| / M, 1) with
    tau > 0 chosen (bisection) so that sum z = k when that is binding; g = 1/2 sum beta_j^2 / z_j."""
    a = np.abs(np.asarray(beta, float))
    lo_z = a / M
    if a.max(initial=0.0) > M or lo_z.sum() > k + 1e-12:
        return math.inf
    nz = a > 0
    if not nz.any():
        return 0.0
    if np.count_nonzero(nz) <= k:
        return 0.5 * float(np.sum(a * a))

    def total(tau):
        return float(np.sum(np.clip(a[nz] / tau, lo_z[nz], 1.0)))

    lo, hi = 1e-300, M
    if total(hi) >= k - 1e-15:  # every z at its lower bound |beta|/M already uses the budget
        tau = hi
    else:
        for _ in range(3000):
            mid = 0.5 * (lo + hi)
            if total(mid) > k:
                lo = mid
            else:
                hi = mid
            if hi - lo <= 1e-16 * hi:
                break
        tau = hi
    z = np.clip(a[nz] / tau, lo_z[nz], 1.0)
    return 0.5 * float(np.sum(a[nz] ** 2 / z))


@pytest.mark.parametrize("seed", range(40))
def test_g_matches_lagrangian_waterfill(seed):
    rng = np.random.default_rng(100 + seed)
    p = int(rng.integers(1, 12))
    k = int(rng.integers(1, p + 2))
    M = float(rng.choice([0.5, 1.0, 3.0]))
    beta = rng.normal(0, 1, size=p)
    beta[rng.random(p) < 0.3] = 0.0
    beta = np.clip(beta, -M, M)
    if np.sum(np.abs(beta)) > k * M:
        beta *= 0.95 * k * M / np.sum(np.abs(beta))
    assert oracle.g_value(beta, k, M) == pytest.approx(g_waterfill(beta, k, M), rel=1e-10, abs=1e-14)


def test_g_special_cases():
    rng = np.random.default_rng(7)
    for _ in range(10):
        beta = rng.normal(size=6)
        beta[[1, 4]] = 0.0
        # ||beta||_0 <= k: g = 1/2 ||beta||^2 (all z_j = 1 on the support)
        assert oracle.g_value(beta, 4, 10.0) == pytest.approx(0.5 * beta @ beta, rel=1e-14)
        # k = 1 (M large): g = 1/2 ||beta||_1^2
        assert oracle.g_value(beta, 1, 100.0) == pytest.approx(0.5 * np.sum(np.abs(beta)) ** 2,
                                                               rel=1e-14)
    # outside the domain
    assert oracle.g_value([3.0, 0.0], 1, 2.0) == math.inf
    assert oracle.g_value([1.5, 1.5, 1.5], 2, 2.0) == math.inf  # ||beta||_1 > k M


@pytest.mark.parametrize("seed", range(20))
def test_gstar_matches_linear_program(seed):
    """Lemma 2's proof: g*(alpha) = max sum H_M(alpha_j) z_j over z in [0,1]^p, 1^T z <= k."""
    rng = np.random.default_rng(200 + seed)
    p = int(rng.integers(1, 15))
    k = int(rng.integers(1, p + 2))
    M = float(rng.choice([0.5, 1.0, 3.0]))
    alpha = rng.normal(0, 2, size=p)
    h = oracle.huber(alpha, M)
    res = linprog(-h, A_ub=np.ones((1, p)), b_ub=[k], bounds=[(0, 1)] * p, method="highs")
    assert oracle.gstar_value(alpha, k, M) == pytest.approx(-res.fun, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("seed", range(40))
def test_fenchel_young_ties_alg1_alg2_lemma2(seed):
    """beta = prox_{g/rho}(x), alpha = prox_{rho g*}(rho x) satisfy x = beta + alpha/rho and
    alpha in dg(beta), hence g(beta) + g*(alpha) = alpha^T beta."""
    rng = np.random.default_rng(300 + seed)
    p = int(rng.integers(1, 40))
    k = int(rng.integers(1, max(2, p // 2 + 1)))
    M = float(rng.choice([0.5, 1.0, 2.0, 20.0]))
    rho = float(rng.choice([0.3, 1.0, 5.0, 200.0]))
    x = rng.normal(0, 1.5, size=p)
    beta = oracle.prox_g(x, rho, M, k)
    alpha = oracle.prox_gstar(rho * x, rho, M, k)
    np.testing.assert_allclose(beta + alpha / rho, x, rtol=1e-12, atol=1e-12)
    lhs = oracle.g_value(beta, k, M, slack=1e-9) + oracle.gstar_value(alpha, k, M)
    rhs = float(alpha @ beta)
    assert lhs == pytest.approx(rhs, rel=1e-9, abs=1e-10)


@pytest.mark.parametrize("seed", range(15))
def test_prox_preserves_magnitude_order(seed):
    rng = np.random.default_rng(400 + seed)
    p = int(rng.integers(2, 200))
    k = int(rng.integers(1, 12))
    x = rng.normal(0, 1, size=p) * rng.choice([0.1, 1.0, 5.0])
    b = oracle.prox_g(x, float(rng.choice([0.5, 2.0, 50.0])), float(rng.choice([0.5, 2.0])), k)
    order = np.argsort(-np.abs(x), kind="stable")
    mags = np.abs(b[order])
    assert np.all(np.diff(mags) <= 1e-12)
    # signs are preserved (or zero, up to the rounding of x - (rho x)/rho in the Moreau identity)
    assert np.all(b * x >= -1e-14 * x * x)


def test_prox_node_parts():
    rng = np.random.default_rng(5)
    p, k, M, rho = 12, 4, 1.0, 2.5
    w = rng.normal(0, 2, size=p)
    ns = oracle.node_sets(p, Z0=[0, 3], Z1=[5, 7])
    beta = oracle.prox_node(w, rho, M, k, ns)
    assert beta[0] == 0.0 and beta[3] == 0.0
    # Z1 coordinates: minimise 1/2 (b - w)^2 + b^2 / (2 rho) over |b| <= M, by golden section
    for j in (5, 7):
        fn = lambda b: 0.5 * (b - w[j]) ** 2 + 0.5 * b * b / rho
        ref = _golden_min(fn, -M, M, iters=200)
        assert beta[j] == pytest.approx(ref, abs=1e-7)  # golden section resolves ~sqrt(eps)
    # free part uses k' = k - |Z1|
    np.testing.assert_allclose(beta[ns.free], oracle.prox_g(w[ns.free], rho, M, k - 2), rtol=1e-15)
    # Fenchel-Young for the node functions
    alpha = rho * (w - beta)
    lhs = oracle.g_node(beta, M, k, ns, slack=1e-9) + oracle.gstar_node(alpha, M, k, ns)
    assert lhs == pytest.approx(float(alpha @ beta), rel=1e-10)
    with pytest.raises(ValueError):
        oracle.node_sets(p, Z0=[1], Z1=[1])
    with pytest.raises(ValueError):
        oracle.node_sets(p, Z0=[p])

"""Plain FP64 CPU oracle for the node relaxation of the k-sparse, box-constrained, ridge GLM.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module. The GPU library never does, and this module imports
nothing from the GPU package.

Source: Liu et al., "Scalable First-order Method for Certifying Optimal k-Sparse GLMs"
(arXiv 2502.09502). Every function names the passage it follows. Everything is IEEE FP64 with
NumPy / SciPy library primitives (matrix products, sorting, a symmetric eigen-solver); there is
no blocking, fusion or reordering beyond what the cited definitions state.

Node form. A branch-and-bound node fixes z_j = 0 on a set Z0 and z_j = 1 on a set Z1 in the
perspective relaxation P_conv (Sec. 2, relaxation of eq. (4)); the free set is F = [p] minus
(Z0 and Z1) and the remaining budget is k' = k - |Z1|. Substituting those z_j in the definition of
g (Sec. 3, eq. (7)) gives the node regulariser

    g_node(beta) = 1/2 sum_{j in Z1} beta_j^2 + g_{k',M}(beta_F)
                   + indicator(beta_{Z0} = 0) + indicator(|beta_j| <= M on Z1),

whose conjugate follows from the separable sum rule (App. D):

    g_node*(alpha) = sum_{j in Z1} H_M(alpha_j) + TopSum_{k'}(H_M(alpha_F)).

|Z1| > k leaves no feasible z: the node is infeasible and its bound is +inf.

Readings of points the paper leaves open (each one is also listed with the design notes):
  * the dual point of the safe bound is zeta = -grad f(X beta_hat) (Sec. 3.4 writes +grad; the
    loss conjugates of App. D.1 need the minus sign for the bound to be finite and tight);
  * least squares is the un-halved, un-normalised sum ||X beta - y||^2 (problem (1), App. D.1);
  * L is the exact Lipschitz constant of grad F: 2 lambda_max(X^T X) for least squares,
    lambda_max(X^T X)/4 for logistic (Alg. 3 only names it);
  * Alg. 3 restarts to phi = 1 and starts from L^1 = f(X 0) + 2 lambda2 g(0) = f(0);
  * the stopping rule is (P_best - D_best) / max(|P_best|, 1) <= tol, checked in FP64;
  * the pooling of Alg. 1 uses a plain block stack, not the up-and-down scan of Alg. 4 (whose
    text is garbled); the isotonic solution is unique (Lemma 3) so the result is the same;
  * sorting ties are broken by ascending index; sgn(0) = 0.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------------------------
# Scalar building blocks (Sec. 3.1, Sec. 3.2)
# ----------------------------------------------------------------------------------------------


def huber(a, M):
    """Huber function H_M of Sec. 3.1, elementwise: a^2/2 if |a| <= M, else M|a| - M^2/2."""
    a = np.abs(np.asarray(a, dtype=np.float64))
    return np.where(a <= M, 0.5 * a * a, M * a - 0.5 * M * M)


def huber_prox_nonneg(c, x, M):
    """argmin_nu 1/2 (nu - x)^2 + c H_M(nu) for x >= 0 and weight c >= 0.

    This is the per-block value of Alg. 1 (initial step, and the pooled step with c = P/N,
    x = S/N as shown in the proof of Lemma 5). Stationarity reads nu - x + c clip(nu, -M, M) = 0:
    the root is x / (1 + c) when that is at most M, and x - c M otherwise.
    """
    if x <= M * (1.0 + c):
        return x / (1.0 + c)
    return x - c * M


# ----------------------------------------------------------------------------------------------
# g*, prox of g*, prox of g, value of g (Lemma 2, Alg. 1, Moreau identity, Alg. 2)
# ----------------------------------------------------------------------------------------------


def gstar_value(alpha, k, M):
    """g*(alpha) = TopSum_k(H_M(alpha)) (Lemma 2). k <= 0 gives 0."""
    h = np.sort(huber(alpha, M))[::-1]
    if k <= 0:
        return 0.0
    return float(np.sum(h[:k]))


def prox_gstar(mu, rho, M, k):
    """prox_{rho g*}(mu) = argmin_alpha 1/2 ||alpha - mu||^2 + rho g*(alpha)  (eq. (10)), by Alg. 1.

    Steps, in the paper's order:
      1. sort |mu| in decreasing order (ties: ascending index);
      2. weights rho_j = rho on the first k sorted positions and 0 after them;
      3. p singleton blocks, each holding its own value argmin 1/2 (nu - |mu_j|)^2 + rho_j H_M(nu);
      4. while two adjacent blocks violate the non-increasing order (left value < right value),
         pool them into one block whose value minimises the block's summed objective, i.e.
         prox_{(P/N) H_M}(S/N) with P = sum of weights, S = sum of |mu|, N = block size;
      5. expand the block values, undo the sort, and multiply by sgn(mu) (Lemma 3).
    """
    mu = np.asarray(mu, dtype=np.float64)
    p = mu.size
    if p == 0:
        return mu.copy()
    order = np.argsort(-np.abs(mu), kind="stable")
    u = np.abs(mu)[order]
    weights = np.where(np.arange(p) < k, float(rho), 0.0)

    blk_P: list[float] = []
    blk_S: list[float] = []
    blk_N: list[int] = []
    blk_V: list[float] = []
    for j in range(p):
        blk_P.append(weights[j])
        blk_S.append(u[j])
        blk_N.append(1)
        blk_V.append(huber_prox_nonneg(weights[j], u[j], M))
        while len(blk_V) > 1 and blk_V[-2] < blk_V[-1]:
            P2, S2, N2 = blk_P.pop(), blk_S.pop(), blk_N.pop()
            blk_V.pop()
            blk_P[-1] += P2
            blk_S[-1] += S2
            blk_N[-1] += N2
            blk_V[-1] = huber_prox_nonneg(blk_P[-1] / blk_N[-1], blk_S[-1] / blk_N[-1], M)

    nu_sorted = np.repeat(np.asarray(blk_V, dtype=np.float64), np.asarray(blk_N))
    nu = np.empty(p, dtype=np.float64)
    nu[order] = nu_sorted
    return np.sign(mu) * nu


def prox_g(x, rho, M, k):
    """prox_{g/rho}(x) by the Moreau identity (Sec. 3.3): x - prox_{rho g*}(rho x) / rho, evaluated
    as (mu - prox_{rho g*}(mu)) / rho with mu = rho x, so that entries the prox of g* leaves
    unchanged (alpha_j = mu_j, e.g. every entry when k = 0) give beta_j = 0 exactly."""
    x = np.asarray(x, dtype=np.float64)
    mu = rho * x
    return (mu - prox_gstar(mu, rho, M, k)) / rho


def in_dom_g(beta, k, M, slack=1e-12):
    """beta is in dom g iff some z of eq. (7) is feasible: ||beta||_inf <= M and ||beta||_1 <= k M.

    A relative slack absorbs FP64 rounding of points produced by the prox.
    """
    a = np.abs(np.asarray(beta, dtype=np.float64))
    if a.size == 0:
        return True
    if k <= 0:
        return bool(np.all(a == 0.0))
    return bool(a.max() <= M * (1.0 + slack) and a.sum() <= k * M * (1.0 + slack))


def g_value(beta, k, M, slack=1e-12):
    """g(beta) of eq. (7) by Alg. 2 (majorisation, Thm. 2); +inf outside dom g.

    Alg. 2: sort |beta| decreasing, s = sum |beta|; for j = 1..k: sbar = s / (k - j + 1); if
    sbar >= |beta_j| set psi_{j..k} = sbar and stop, else psi_j = |beta_j| and s -= |beta_j|;
    return 1/2 ||psi||^2. When k exceeds p, |beta| is padded with zeros.
    """
    beta = np.asarray(beta, dtype=np.float64)
    if not in_dom_g(beta, k, M, slack):
        return math.inf
    if k <= 0:
        return 0.0
    a = np.sort(np.abs(beta))[::-1]
    s = float(np.sum(a))
    psi = np.zeros(k, dtype=np.float64)
    for j in range(k):
        bj = a[j] if j < a.size else 0.0
        sbar = s / (k - j)
        if sbar >= bj:
            psi[j:] = sbar
            break
        psi[j] = bj
        s -= bj
    return 0.5 * float(np.sum(psi * psi))


# ----------------------------------------------------------------------------------------------
# Node forms (z fixed on Z0 / Z1)
# ----------------------------------------------------------------------------------------------


@dataclass
class NodeSets:
    """Index sets of one node. zero = Z0 (z_j = 0), one = Z1 (z_j = 1), free = F."""

    p: int
    zero: np.ndarray
    one: np.ndarray
    free: np.ndarray

    @property
    def kprime_offset(self) -> int:
        return int(self.one.size)


def node_sets(p, Z0=(), Z1=()):
    """Validate the fixed sets (0-based, no duplicates, in range, disjoint) and build F."""
    Z0 = np.asarray(sorted(int(j) for j in Z0), dtype=np.int64)
    Z1 = np.asarray(sorted(int(j) for j in Z1), dtype=np.int64)
    for Z in (Z0, Z1):
        if Z.size and (Z.min() < 0 or Z.max() >= p):
            raise ValueError("fixed index out of range")
        if np.unique(Z).size != Z.size:
            raise ValueError("duplicate fixed index")
    if np.intersect1d(Z0, Z1).size:
        raise ValueError("an index is fixed both to zero and to one")
    mask = np.ones(p, dtype=bool)
    mask[Z0] = False
    mask[Z1] = False
    return NodeSets(p=p, zero=Z0, one=Z1, free=np.nonzero(mask)[0])


def prox_node(w, rho, M, k, ns: NodeSets):
    """prox_{g_node/rho}(w) = argmin_beta 1/2 ||beta - w||^2 + g_node(beta)/rho.

    The node regulariser is separable over (Z0, Z1, F):
      Z0: beta_j = 0;
      Z1: argmin 1/2 (b - w_j)^2 + b^2/(2 rho) over |b| <= M, i.e. clip(rho w_j / (1 + rho), -M, M);
      F : prox_{g_{k'}/rho}(w_F) by the Moreau identity and Alg. 1 with k' = k - |Z1|.
    """
    w = np.asarray(w, dtype=np.float64)
    kp = k - ns.one.size
    if kp < 0:
        raise ValueError("infeasible node: |Z1| > k")
    beta = np.zeros_like(w)
    if ns.one.size:
        beta[ns.one] = np.clip(rho * w[ns.one] / (1.0 + rho), -M, M)
    if ns.free.size:
        beta[ns.free] = prox_g(w[ns.free], rho, M, kp)
    return beta


def g_node(beta, M, k, ns: NodeSets, slack=1e-12):
    """g_node(beta) (see the module docstring); +inf outside its domain."""
    beta = np.asarray(beta, dtype=np.float64)
    kp = k - ns.one.size
    if kp < 0:
        return math.inf
    if ns.zero.size and np.any(beta[ns.zero] != 0.0):
        return math.inf
    b1 = beta[ns.one]
    if b1.size and np.max(np.abs(b1)) > M * (1.0 + slack):
        return math.inf
    return 0.5 * float(np.sum(b1 * b1)) + g_value(beta[ns.free], kp, M, slack)


def gstar_node(alpha, M, k, ns: NodeSets):
    """g_node*(alpha) = sum_{Z1} H_M(alpha_j) + TopSum_{k'}(H_M(alpha_F)); Z0 contributes 0."""
    alpha = np.asarray(alpha, dtype=np.float64)
    kp = k - ns.one.size
    return float(np.sum(huber(alpha[ns.one], M))) + gstar_value(alpha[ns.free], kp, M)


# ----------------------------------------------------------------------------------------------
# GLM losses and their conjugates (problem (1), App. D.1)
# ----------------------------------------------------------------------------------------------


def _xlogx(q):
    q = np.asarray(q, dtype=np.float64)
    out = np.zeros_like(q)
    pos = q > 0
    out[pos] = q[pos] * np.log(q[pos])
    return out


class LeastSquares:
    """f(u, y) = ||u - y||^2; F*(-zeta) = ||zeta||^2 / 4 - y^T zeta (App. D.1)."""

    name = "ls"

    @staticmethod
    def f(u, y):
        r = np.asarray(u, dtype=np.float64) - y
        return float(r @ r)

    @staticmethod
    def grad(u, y):
        return 2.0 * (np.asarray(u, dtype=np.float64) - y)

    @staticmethod
    def conj_neg(zeta, y):
        zeta = np.asarray(zeta, dtype=np.float64)
        return 0.25 * float(zeta @ zeta) - float(y @ zeta)

    @staticmethod
    def lipschitz_factor():
        return 2.0


class Logistic:
    """f(u, y) = sum log(1 + exp(-y_i u_i)), y in {-1, +1};
    F*(-zeta) = sum (1 - q_i) log(1 - q_i) + q_i log q_i with q_i = zeta_i / y_i in [0, 1] (App. D.1),
    +inf when some q_i leaves [0, 1]."""

    name = "logistic"

    @staticmethod
    def f(u, y):
        return float(np.sum(np.logaddexp(0.0, -y * np.asarray(u, dtype=np.float64))))

    @staticmethod
    def grad(u, y):
        # d/du log(1 + exp(-y u)) = -y sigmoid(-y u)
        t = -y * np.asarray(u, dtype=np.float64)
        return -y * _sigmoid(t)

    @staticmethod
    def conj_neg(zeta, y, slack=1e-15):
        q = np.asarray(zeta, dtype=np.float64) * y  # zeta / y for y = +-1
        if np.any(q < -slack) or np.any(q > 1.0 + slack):
            return math.inf
        q = np.clip(q, 0.0, 1.0)
        return float(np.sum(_xlogx(q) + _xlogx(1.0 - q)))

    @staticmethod
    def lipschitz_factor():
        return 0.25


class SquaredHinge:
    """f(u, y) = sum max(0, 1 - y_i u_i)^2, y in {-1, +1};
    F*(-zeta) = sum h(-y_i zeta_i) with h(z) = z + z^2/4 for z <= 0 and +inf for z > 0
    (App. D.1). The derivative -2 y max(0, 1 - y u) is 2-Lipschitz in u."""

    name = "sqhinge"

    @staticmethod
    def f(u, y):
        m = np.maximum(0.0, 1.0 - y * np.asarray(u, dtype=np.float64))
        return float(m @ m)

    @staticmethod
    def grad(u, y):
        return -2.0 * y * np.maximum(0.0, 1.0 - y * np.asarray(u, dtype=np.float64))

    @staticmethod
    def conj_neg(zeta, y, slack=1e-15):
        z = -y * np.asarray(zeta, dtype=np.float64)
        if np.any(z > slack):
            return math.inf
        z = np.minimum(z, 0.0)
        return float(np.sum(z + 0.25 * z * z))

    @staticmethod
    def lipschitz_factor():
        return 2.0


def _h_entropy(z):
    """h(z) = z log z - z for z > 0, h(0) = 0, +inf for z < 0 (App. D.1)."""
    z = np.asarray(z, dtype=np.float64)
    if np.any(z < 0):
        return math.inf
    return float(np.sum(_xlogx(z) - z))


class Poisson:
    """f(u, y) = sum exp(u_i) - y_i u_i, y_i >= 0; F*(-zeta) = sum h(y_i - zeta_i) (App. D.1).
    The derivative exp(u) - y has no global Lipschitz constant: L must be supplied."""

    name = "poisson"

    @staticmethod
    def f(u, y):
        u = np.asarray(u, dtype=np.float64)
        return float(np.sum(np.exp(u) - y * u))

    @staticmethod
    def grad(u, y):
        return np.exp(np.asarray(u, dtype=np.float64)) - y

    @staticmethod
    def conj_neg(zeta, y):
        return _h_entropy(y - np.asarray(zeta, dtype=np.float64))

    @staticmethod
    def lipschitz_factor():
        raise ValueError("the Poisson loss has no global Lipschitz constant; give L")


class Gamma:
    """f(u, y) = sum y_i exp(-u_i) + u_i, y_i > 0. Its conjugate, from the definition:
    f_i*(s) = sup_u (s - 1) u - y_i exp(-u) = y_i h((1 - s) / y_i), so F*(-zeta) =
    sum y_i h((1 + zeta_i) / y_i) (App. D.1 prints the argument with the other sign of zeta).
    The derivative 1 - y exp(-u) has no global Lipschitz constant: L must be supplied."""

    name = "gamma"

    @staticmethod
    def f(u, y):
        u = np.asarray(u, dtype=np.float64)
        return float(np.sum(y * np.exp(-u) + u))

    @staticmethod
    def grad(u, y):
        return 1.0 - y * np.exp(-np.asarray(u, dtype=np.float64))

    @staticmethod
    def conj_neg(zeta, y):
        z = (1.0 + np.asarray(zeta, dtype=np.float64)) / y
        if np.any(z < 0):
            return math.inf
        return float(np.sum(y * (_xlogx(z) - z)))

    @staticmethod
    def lipschitz_factor():
        raise ValueError("the Gamma loss has no global Lipschitz constant; give L")


def _sigmoid(t):
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    pos = t >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-t[pos]))
    e = np.exp(t[~pos])
    out[~pos] = e / (1.0 + e)
    return out


LOSSES = {"ls": LeastSquares, "logistic": Logistic, "sqhinge": SquaredHinge,
          "poisson": Poisson, "gamma": Gamma}


def get_loss(loss):
    if isinstance(loss, str):
        return LOSSES[loss]
    return loss


# ----------------------------------------------------------------------------------------------
# Objective, dual bound, Lipschitz constant (Sec. 3.3, Sec. 3.4)
# ----------------------------------------------------------------------------------------------


def primal_value(X, y, loss, lam2, M, k, ns: NodeSets, beta):
    """Objective of eq. (6) at a node: f(X beta) + 2 lambda2 g_node(beta)."""
    loss = get_loss(loss)
    gv = g_node(beta, M, k, ns)
    if math.isinf(gv):
        return math.inf
    return loss.f(X @ beta, y) + 2.0 * lam2 * gv


def dual_value(X, y, loss, lam2, M, k, ns: NodeSets, zeta):
    """Weak-duality bound of Sec. 3.4: D(zeta) = -F*(-zeta) - G*(X^T zeta), valid for every zeta.

    G = 2 lambda2 g_node, so G*(v) = 2 lambda2 g_node*(v / (2 lambda2)) (scalar multiplication rule,
    App. D).
    """
    loss = get_loss(loss)
    v = X.T @ zeta
    fc = loss.conj_neg(zeta, y)
    if math.isinf(fc):
        return -math.inf
    return -fc - 2.0 * lam2 * gstar_node(v / (2.0 * lam2), M, k, ns)


def lambda_max_gram(X):
    """Largest eigenvalue of X^T X. Dense symmetric eigen-solver for p <= 2000, else Lanczos."""
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    if p <= 2000:
        return float(np.linalg.eigvalsh(X.T @ X)[-1])
    from scipy.sparse.linalg import LinearOperator, eigsh

    op = LinearOperator((p, p), matvec=lambda v: X.T @ (X @ v), dtype=np.float64)
    vals = eigsh(op, k=1, which="LA", tol=1e-12, return_eigenvectors=False)
    return float(vals[0])


def lipschitz(X, loss):
    """Lipschitz constant of grad F(beta) = X^T grad f(X beta): 2 lambda_max for least squares
    (Hessian 2 X^T X), lambda_max / 4 for logistic (sigmoid' <= 1/4)."""
    return get_loss(loss).lipschitz_factor() * lambda_max_gram(X)


# ----------------------------------------------------------------------------------------------
# Restarted FISTA (Alg. 3) with the FP64 certificate
# ----------------------------------------------------------------------------------------------

CONVERGED = "converged"
NOT_CONVERGED = "not_converged"
INFEASIBLE = "infeasible"


@dataclass
class NodeResult:
    beta: np.ndarray
    primal: float
    lower_bound: float
    gap_abs: float
    gap_rel: float
    iters: int
    restarts: int
    status: str
    L: float = float("nan")
    history: list = field(default_factory=list)


def rel_gap(P, D):
    return (P - D) / max(abs(P), 1.0)


def solve_node(X, y, loss, lam2, M, k, Z0=(), Z1=(), tol=1e-6, max_iter=100000, check_every=1,
               L=None, warm_start=None, restart=True, momentum=True, record=False):
    """Solve the node relaxation by Alg. 3 and certify it with the bound of Sec. 3.4.

    Alg. 3, for t = 1, 2, ...:
      gamma   = beta^t + phi/(phi + 3) (beta^t - beta^{t-1})          (momentum)
      gamma   = gamma - grad F(gamma) / L,  grad F(b) = X^T grad f(X b)
      beta^{t+1} = prox_{g_node/rho}(gamma),  rho = L / (2 lambda2)   (Moreau identity + Alg. 1)
      L^{t+1} = f(X beta^{t+1}) + 2 lambda2 g_node(beta^{t+1})         (Alg. 2)
      phi     = 1 if L^{t+1} >= L^t else phi + 1                       (restart)
    Every check_every iterations: zeta = -grad f(X beta^{t+1}), D = D(zeta); keep the best primal
    P (and its beta) and the best D; stop when (P - D) / max(|P|, 1) <= tol.

    restart=False keeps phi growing (plain FISTA); momentum=False uses phi/(phi+3) = 0 (PGD).
    """
    loss = get_loss(loss)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, p = X.shape
    if y.shape != (n,):
        raise ValueError("y must have n entries")
    if not (lam2 > 0 and M > 0 and k >= 1):
        raise ValueError("need lambda2 > 0, M > 0, k >= 1")
    if not (np.all(np.isfinite(X)) and np.all(np.isfinite(y))):
        raise ValueError("non-finite data")
    if loss is Logistic and not np.all(np.abs(y) == 1.0):
        raise ValueError("logistic labels must be -1 or +1")
    ns = node_sets(p, Z0, Z1)
    if ns.one.size > k:
        return NodeResult(beta=np.zeros(p), primal=math.inf, lower_bound=math.inf, gap_abs=0.0,
                          gap_rel=0.0, iters=0, restarts=0, status=INFEASIBLE)
    if L is None:
        L = lipschitz(X, loss)
    rho = L / (2.0 * lam2)

    beta = np.zeros(p)
    if warm_start is not None:
        beta = np.asarray(warm_start, dtype=np.float64).copy()
        beta[ns.zero] = 0.0
    beta_prev = beta.copy()
    phi = 1.0
    L_prev = primal_value(X, y, loss, lam2, M, k, ns, beta)
    P_best, beta_best = L_prev, beta.copy()
    D_best = -math.inf
    restarts = 0
    history = []
    status = NOT_CONVERGED
    t = 0
    for t in range(1, max_iter + 1):
        c = phi / (phi + 3.0) if momentum else 0.0
        gamma = beta + c * (beta - beta_prev)
        grad = X.T @ loss.grad(X @ gamma, y)
        w = gamma - grad / L
        beta_new = prox_node(w, rho, M, k, ns)
        L_new = primal_value(X, y, loss, lam2, M, k, ns, beta_new)
        if restart and L_new >= L_prev:
            phi = 1.0
            restarts += 1
        else:
            phi += 1.0
        beta_prev, beta = beta, beta_new
        L_prev = L_new
        if L_new < P_best:
            P_best, beta_best = L_new, beta_new.copy()
        if t % check_every == 0:
            zeta = -loss.grad(X @ beta_new, y)
            D = dual_value(X, y, loss, lam2, M, k, ns, zeta)
            D_best = max(D_best, D)
            if record:
                history.append((t, L_new, D, P_best, D_best))
            if rel_gap(P_best, D_best) <= tol:
                status = CONVERGED
                break
    return NodeResult(beta=beta_best, primal=P_best, lower_bound=D_best,
                      gap_abs=P_best - D_best, gap_rel=rel_gap(P_best, D_best), iters=t,
                      restarts=restarts, status=status, L=L, history=history)


# ----------------------------------------------------------------------------------------------
# Eigen-perspective relaxation for least squares (App. D.2)
# ----------------------------------------------------------------------------------------------
#
# With Q = X^T X - s I (0 <= s <= lambda_min(X^T X), so Q is positive semidefinite) and
# lambda_eig = lambda2 + s, the node problem's least-squares objective splits as
#   ||X b - y||^2 + lambda2 sum b_j^2 / z_j = b^T Q b - 2 y^T X b + ||y||^2 + s ||b||^2 + ...,
# and s ||b||^2 + lambda2 sum b_j^2 / z_j <= lambda_eig sum b_j^2 / z_j for z in [0, 1], so
#   P_eig(node) = min_b  b^T Q b - 2 y^T X b + ||y||^2 + 2 lambda_eig g_node(b)
# lies between the perspective relaxation and P_MIP (s = 0 gives the perspective relaxation).
# Weak duality with F(b) = b^T Q b and G(b) = -2 y^T X b + 2 lambda_eig g_node(b) at
# zeta = -grad F(b_hat) = -2 Q b_hat gives (the constant ||y||^2 kept so that the bound is one of
# the node's objective; App. D.2 drops it, and its last display has the signs of both terms
# flipped):
#   D_eig(b_hat) = ||y||^2 - b_hat^T Q b_hat - 2 lambda_eig g_node*((X^T y - Q b_hat) / lambda_eig).


def lambda_min_gram(X):
    """Smallest eigenvalue of X^T X (dense symmetric eigen-solver for p <= 2000, else Lanczos)."""
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    if p <= 2000:
        return float(np.linalg.eigvalsh(X.T @ X)[0])
    from scipy.sparse.linalg import LinearOperator, eigsh

    op = LinearOperator((p, p), matvec=lambda v: X.T @ (X @ v), dtype=np.float64)
    return float(eigsh(op, k=1, which="SA", tol=1e-12, return_eigenvectors=False)[0])


def eig_primal_value(X, y, lam2, M, k, ns: NodeSets, beta, shift):
    """Objective of the eigen-perspective node problem: ||X b - y||^2 - s ||b||^2
    + 2 (lambda2 + s) g_node(b)."""
    gv = g_node(beta, M, k, ns)
    if math.isinf(gv):
        return math.inf
    r = X @ beta - y
    return float(r @ r) - shift * float(beta @ beta) + 2.0 * (lam2 + shift) * gv


def eig_dual_value(X, y, lam2, M, k, ns: NodeSets, beta_hat, shift):
    """D_eig(b_hat) above: ||y||^2 - b^T Q b - 2 lambda_eig g_node*((X^T y - Q b) / lambda_eig)."""
    lam_eig = lam2 + shift
    Qb = X.T @ (X @ beta_hat) - shift * beta_hat
    a = (X.T @ y - Qb) / lam_eig
    return float(y @ y) - float(beta_hat @ Qb) - 2.0 * lam_eig * gstar_node(a, M, k, ns)


def solve_node_eig(X, y, lam2, M, k, shift, Z0=(), Z1=(), tol=1e-6, max_iter=100000, L=None):
    """Alg. 3 on the eigen-perspective node problem (least squares), certified by D_eig:
      gamma = beta^t + phi/(phi+3) (beta^t - beta^{t-1});
      grad  = 2 Q gamma - 2 X^T y = X^T (2 (X gamma - y)) - 2 s gamma;
      beta^{t+1} = prox_{g_node / rho}(gamma - grad / L), rho = L / (2 lambda_eig),
      L = 2 lambda_max(Q) = 2 (lambda_max(X^T X) - s);
      restart on the objective, and D_eig(beta^{t+1}) every iteration."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, p = X.shape
    if not (0.0 <= shift):
        raise ValueError("the shift must be >= 0")
    ns = node_sets(p, Z0, Z1)
    if ns.one.size > k:
        return NodeResult(beta=np.zeros(p), primal=math.inf, lower_bound=math.inf, gap_abs=0.0,
                          gap_rel=0.0, iters=0, restarts=0, status=INFEASIBLE)
    if L is None:
        L = 2.0 * (lambda_max_gram(X) - shift)
    lam_eig = lam2 + shift
    rho = L / (2.0 * lam_eig)
    beta = np.zeros(p)
    beta_prev = beta.copy()
    phi = 1.0
    L_prev = eig_primal_value(X, y, lam2, M, k, ns, beta, shift)
    P_best, beta_best = L_prev, beta.copy()
    D_best = -math.inf
    restarts = 0
    status = NOT_CONVERGED
    t = 0
    for t in range(1, max_iter + 1):
        c = phi / (phi + 3.0)
        gamma = beta + c * (beta - beta_prev)
        grad = X.T @ (2.0 * (X @ gamma - y)) - 2.0 * shift * gamma
        beta_new = prox_node(gamma - grad / L, rho, M, k, ns)
        L_new = eig_primal_value(X, y, lam2, M, k, ns, beta_new, shift)
        if L_new >= L_prev:
            phi = 1.0
            restarts += 1
        else:
            phi += 1.0
        beta_prev, beta = beta, beta_new
        L_prev = L_new
        if L_new < P_best:
            P_best, beta_best = L_new, beta_new.copy()
        D_best = max(D_best, eig_dual_value(X, y, lam2, M, k, ns, beta_new, shift))
        if rel_gap(P_best, D_best) <= tol:
            status = CONVERGED
            break
    return NodeResult(beta=beta_best, primal=P_best, lower_bound=D_best,
                      gap_abs=P_best - D_best, gap_rel=rel_gap(P_best, D_best), iters=t,
                      restarts=restarts, status=status, L=L)


# ----------------------------------------------------------------------------------------------
# Brute-force mixed-integer optimum for tiny p (tests only)
# ----------------------------------------------------------------------------------------------


def _box_ridge_ls(XS, y, lam2, M):
    """min ||XS b - y||^2 + lam2 ||b||^2 over |b_j| <= M, exactly: each coordinate is free, at +M or
    at -M; solve the free part, keep the pattern that satisfies the KKT conditions."""
    s = XS.shape[1]
    if s == 0:
        return float(y @ y), np.zeros(0)
    Q = XS.T @ XS + lam2 * np.eye(s)
    q = XS.T @ y
    best = (math.inf, None)
    for pattern in itertools.product((0, 1, -1), repeat=s):
        pat = np.asarray(pattern)
        b = np.zeros(s)
        fixed = pat != 0
        b[fixed] = M * pat[fixed]
        free = ~fixed
        if free.any():
            rhs = q[free] - Q[np.ix_(free, fixed)] @ b[fixed]
            b[free] = np.linalg.solve(Q[np.ix_(free, free)], rhs)
            if np.any(np.abs(b[free]) > M * (1 + 1e-12)):
                continue
        gradient = 2.0 * (Q @ b - q)  # gradient of the objective
        ok = True
        for j in np.nonzero(fixed)[0]:
            # at +M the gradient must be <= 0, at -M it must be >= 0
            if pat[j] > 0 and gradient[j] > 1e-9 * max(1.0, abs(q[j])):
                ok = False
            if pat[j] < 0 and gradient[j] < -1e-9 * max(1.0, abs(q[j])):
                ok = False
        if not ok:
            continue
        r = XS @ b - y
        val = float(r @ r + lam2 * b @ b)
        if val < best[0]:
            best = (val, b)
    return best


def _box_ridge_smooth(XS, y, lam2, M, loss):
    """min_{|b|_inf <= M} f(XS b) + lambda2 ||b||^2 for a smooth loss (L-BFGS-B with bounds)."""
    from scipy.optimize import minimize

    s = XS.shape[1]
    if s == 0:
        return loss.f(np.zeros(len(y)), y), np.zeros(0)

    def fun(b):
        u = XS @ b
        return loss.f(u, y) + lam2 * b @ b, XS.T @ loss.grad(u, y) + 2 * lam2 * b

    res = minimize(fun, np.zeros(s), jac=True, method="L-BFGS-B", bounds=[(-M, M)] * s,
                   options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 10000})
    return float(res.fun), res.x


def brute_force_mip(X, y, loss, lam2, M, k, Z0=(), Z1=()):
    """P_MIP of the node (eq. (4) with z fixed on Z0 / Z1): the minimum over supports S with
    Z1 in S, S in Z1 union F, |S| <= k of min_{|b|_inf <= M} f(X_S b) + lambda2 ||b||^2.
    Exponential in p; for p <= 12, k <= 3."""
    loss = get_loss(loss)
    X = np.asarray(X, dtype=np.float64)
    p = X.shape[1]
    ns = node_sets(p, Z0, Z1)
    if ns.one.size > k:
        return math.inf
    solver = _box_ridge_ls if loss is LeastSquares else (
        lambda XS, yy, l2, MM: _box_ridge_smooth(XS, yy, l2, MM, loss))
    best = math.inf
    for extra in range(0, k - ns.one.size + 1):
        for comb in itertools.combinations(ns.free.tolist(), extra):
            S = np.asarray(sorted(ns.one.tolist() + list(comb)), dtype=np.int64)
            val, _ = solver(X[:, S], y, lam2, M)
            best = min(best, val)
    return best

"""FP64 CPU oracle (test infrastructure only; see ``oracle.core``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package. It shares no code with the GPU library.
"""
from .core import (  # noqa: F401
    CONVERGED,
    INFEASIBLE,
    NOT_CONVERGED,
    LeastSquares,
    Logistic,
    SquaredHinge,
    Poisson,
    Gamma,
    NodeResult,
    NodeSets,
    brute_force_mip,
    dual_value,
    g_node,
    g_value,
    get_loss,
    gstar_node,
    gstar_value,
    huber,
    huber_prox_nonneg,
    in_dom_g,
    lambda_max_gram,
    lipschitz,
    node_sets,
    primal_value,
    prox_g,
    prox_gstar,
    prox_node,
    rel_gap,
    solve_node,
)

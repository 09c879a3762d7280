"""ctypes binding of libcertglm.so: argument marshalling only; every step of the solve runs in
the library's HIP kernels. The binding never falls back to a CPU implementation: when the
library is missing it raises."""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcertglm.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_BUSY, E_NOTFOUND, E_INTERNAL = range(7)
F64, F32, BF16 = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
LOSS = {"ls": 0, "logistic": 1, "sqhinge": 2, "poisson": 3, "gamma": 4}
PREC = {"f64": 0, "mixed": 1}
STATUS = {0: "converged", 1: "not_converged", 2: "infeasible", 3: "numeric", 4: "cancelled",
          5: "pruned", 6: "below_incumbent"}

EXPORTS = [
    "cgl_version", "cgl_status_str", "cgl_last_error", "cgl_node_init", "cgl_ctx_create",
    "cgl_ctx_destroy", "cgl_ctx_set_profiling", "cgl_ctx_kernel_stats", "cgl_problem_create", "cgl_problem_destroy", "cgl_problem_lipschitz",
    "cgl_node_validate", "cgl_solve_node", "cgl_solve_batch", "cgl_solve_batch_dual",
    "cgl_certify", "cgl_problem_matvec",
    "cgl_prox_node_batch", "cgl_prox_batch_noalloc", "cgl_problem_set_eigen",
    "cgl_problem_eigen_shift", "cgl_problem_share_design", "cgl_server_create", "cgl_server_submit", "cgl_server_poll",
    "cgl_server_cancel", "cgl_server_stats", "cgl_server_destroy",
]


class CglNode(C.Structure):
    _fields_ = [
        ("fixed_zero", C.POINTER(C.c_int32)), ("n_zero", C.c_int32),
        ("fixed_in", C.POINTER(C.c_int32)), ("n_in", C.c_int32),
        ("tol", C.c_double), ("max_iter", C.c_int32), ("check_every", C.c_int32),
        ("precision", C.c_int32), ("warm_start", C.POINTER(C.c_double)),
        ("incumbent", C.c_double),
    ]


class CglResult(C.Structure):
    _fields_ = [
        ("lower_bound", C.c_double), ("primal", C.c_double), ("gap_abs", C.c_double),
        ("gap_rel", C.c_double), ("iters", C.c_int32), ("restarts", C.c_int32),
        ("status", C.c_int32), ("recentres", C.c_int32), ("err_vs_fp64_est", C.c_double),
    ]


class CglError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is not built; run paper_2502_09502_amd/build.py")
    lib = C.CDLL(path)
    P, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pd = C.POINTER(C.c_double)
    lib.cgl_version.restype = C.c_int
    lib.cgl_status_str.restype = C.c_char_p
    lib.cgl_status_str.argtypes = [C.c_int]
    lib.cgl_last_error.restype = C.c_char_p
    lib.cgl_node_init.argtypes = [C.POINTER(CglNode)]
    lib.cgl_node_init.restype = None
    lib.cgl_ctx_create.argtypes = [C.c_int, P, C.POINTER(P)]
    lib.cgl_ctx_destroy.argtypes = [P]
    lib.cgl_ctx_set_profiling.argtypes = [P, i32]
    lib.cgl_ctx_kernel_stats.argtypes = [P, i32, i32, pd, C.POINTER(i64)]
    lib.cgl_problem_create.argtypes = [P, P, i32, i32, i64, i64, i64, pd, i32, dbl, dbl, i32, dbl,
                                       C.POINTER(P)]
    lib.cgl_problem_destroy.argtypes = [P]
    lib.cgl_problem_lipschitz.argtypes = [P, pd]
    lib.cgl_solve_node.argtypes = [P, C.POINTER(CglNode), pd, C.POINTER(CglResult)]
    lib.cgl_solve_batch.argtypes = [P, C.POINTER(CglNode), i32, pd, C.POINTER(CglResult)]
    lib.cgl_solve_batch_dual.argtypes = [P, C.POINTER(CglNode), i32, pd, C.POINTER(CglResult),
                                         pd]
    lib.cgl_node_validate.argtypes = [C.POINTER(CglNode), i64, i32, C.POINTER(i32)]
    lib.cgl_certify.argtypes = [P, C.POINTER(CglNode), pd, pd, pd]
    lib.cgl_problem_matvec.argtypes = [P, i32, pd, pd]
    lib.cgl_prox_node_batch.argtypes = [P, dbl, dbl, i32, C.POINTER(CglNode), pd, i32, i64, pd, pd]
    lib.cgl_prox_batch_noalloc.argtypes = [P, dbl, dbl, i32, P, i32, i64, P, P]
    lib.cgl_problem_set_eigen.argtypes = [P, dbl]
    lib.cgl_problem_eigen_shift.argtypes = [P, pd]
    lib.cgl_problem_share_design.argtypes = [P, P]
    if hasattr(lib, "cgl_server_create"):
        lib.cgl_server_create.argtypes = [P, C.c_size_t, i32, C.POINTER(P)]
        lib.cgl_server_submit.argtypes = [P, P, C.POINTER(CglNode), C.POINTER(C.c_uint64)]
        lib.cgl_server_poll.argtypes = [P, i32, C.POINTER(C.c_uint64), C.POINTER(CglResult), pd,
                                        i64, pd, C.POINTER(i32)]
        lib.cgl_server_cancel.argtypes = [P, C.c_uint64]
        lib.cgl_server_stats.argtypes = [P, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        lib.cgl_server_destroy.argtypes = [P]
    _lib = lib
    return lib


def check(code):
    if code != OK:
        lib = load()
        raise CglError(code, lib.cgl_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Context:
    def __init__(self, device: int = 0, stream=None):
        self.lib = load()
        self.h = C.c_void_p()
        check(self.lib.cgl_ctx_create(device, stream, C.byref(self.h)))

    def close(self):
        if self.h:
            self.lib.cgl_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def set_profiling(self, on: bool, x_pass: bool = False, phases_only: bool = False):
        """Kernel timing on or off; x_pass also times the batched X pass (level 2);
        phases_only records only the batched engine's phase wall times (level 3, graphs on)."""
        level = 0 if not on else (3 if phases_only else (2 if x_pass else 1))
        check(self.lib.cgl_ctx_set_profiling(self.h, level))

    def kernel_stats(self, which: int, reset: bool = False):
        """(total milliseconds, launches) of one timed kernel (see cgl_ctx_kernel_stats)."""
        ms, n = C.c_double(), C.c_int64()
        check(self.lib.cgl_ctx_kernel_stats(self.h, which, 1 if reset else 0, C.byref(ms),
                                            C.byref(n)))
        return ms.value, n.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Result:
    lower_bound: float
    primal: float
    gap_abs: float
    gap_rel: float
    iters: int
    restarts: int
    status: str
    recentres: int
    err_vs_fp64_est: float
    beta: np.ndarray | None = None


def _result(r: CglResult, beta=None) -> Result:
    return Result(r.lower_bound, r.primal, r.gap_abs, r.gap_rel, r.iters, r.restarts,
                  STATUS.get(r.status, str(r.status)), r.recentres, r.err_vs_fp64_est, beta)


class NodeSpec:
    """Holds a CglNode together with the arrays it points to."""

    def __init__(self, p, Z0=(), Z1=(), tol=1e-6, max_iter=100000, check_every=1,
                 precision="f64", warm_start=None, incumbent=math.inf):
        self.z0 = np.ascontiguousarray(np.asarray(Z0, dtype=np.int32).reshape(-1))
        self.z1 = np.ascontiguousarray(np.asarray(Z1, dtype=np.int32).reshape(-1))
        self.ws = None if warm_start is None else np.ascontiguousarray(warm_start, dtype=np.float64)
        c = CglNode()
        load().cgl_node_init(C.byref(c))
        c.fixed_zero = self.z0.ctypes.data_as(C.POINTER(C.c_int32)) if self.z0.size else None
        c.n_zero = int(self.z0.size)
        c.fixed_in = self.z1.ctypes.data_as(C.POINTER(C.c_int32)) if self.z1.size else None
        c.n_in = int(self.z1.size)
        c.tol = float(tol)
        c.max_iter = int(max_iter)
        c.check_every = int(check_every)
        c.precision = PREC[precision] if isinstance(precision, str) else int(precision)
        c.warm_start = _dptr(self.ws) if self.ws is not None else None
        c.incumbent = float(incumbent)
        self.c = c


class Problem:
    """A problem (X, y, loss, lambda2, M, k) resident on the device.

    X: numpy array (float64, float32, or uint16 bfloat16 patterns), or a C-contiguous array in
    device memory of one of those dtypes (a devmem.DeviceArray; then no host copy is made)."""

    def __init__(self, ctx: Context, X, y, loss="ls", lam2=1e-3, M=2.0, k=10, L=0.0):
        self.ctx = ctx
        self.lib = ctx.lib
        mem = MEM_HOST
        if hasattr(X, "data_ptr"):  # device memory
            dt = {np.dtype(np.float64): F64, np.dtype(np.float32): F32,
                  np.dtype(np.uint16): BF16}[np.dtype(X.dtype)]
            n, p = X.shape
            ptr = C.c_void_p(X.data_ptr())
            mem = MEM_DEVICE
            self._keep = X
        else:
            X = np.ascontiguousarray(X)
            dt = {np.dtype(np.float64): F64, np.dtype(np.float32): F32,
                  np.dtype(np.uint16): BF16}[X.dtype]
            n, p = X.shape
            ptr = X.ctypes.data_as(C.c_void_p)
            self._keep = X
        y = np.ascontiguousarray(y, dtype=np.float64)
        self.n, self.p = int(n), int(p)
        self.h = C.c_void_p()
        check(self.lib.cgl_problem_create(ctx.h, ptr, dt, mem, n, p, p, _dptr(y), LOSS[loss],
                                          float(lam2), float(M), int(k), float(L),
                                          C.byref(self.h)))
        self._keep = None

    def close(self):
        if self.h:
            self.lib.cgl_problem_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def L(self) -> float:
        v = C.c_double()
        check(self.lib.cgl_problem_lipschitz(self.h, C.byref(v)))
        return v.value

    def set_eigen(self, shift: float) -> None:
        """Eigen-perspective relaxation with Q = X^T X - shift I (0 <= shift <= lambda_min)."""
        check(self.lib.cgl_problem_set_eigen(self.h, float(shift)))

    def eigen_shift(self) -> float:
        """The largest shift the library's Cholesky test proves (<= lambda_min(X^T X))."""
        v = C.c_double()
        check(self.lib.cgl_problem_eigen_shift(self.h, C.byref(v)))
        return v.value

    def share_design(self, other: "Problem") -> None:
        """Serve other's mixed-precision nodes from this problem's batched engine (same X)."""
        check(self.lib.cgl_problem_share_design(self.h, other.h))

    def node(self, **kw) -> NodeSpec:
        return NodeSpec(self.p, **kw)

    def solve(self, Z0=(), Z1=(), **kw) -> Result:
        spec = NodeSpec(self.p, Z0=Z0, Z1=Z1, **kw)
        beta = np.empty(self.p)
        r = CglResult()
        check(self.lib.cgl_solve_node(self.h, C.byref(spec.c), _dptr(beta), C.byref(r)))
        return _result(r, beta)

    def solve_batch(self, specs: list[NodeSpec], out=None) -> list[Result]:
        """Solves the nodes together. out: optional C-contiguous float64 array (len(specs), p)
        that receives the solutions (a caller's persistent buffer); the results' beta arrays are
        its rows."""
        arr = (CglNode * len(specs))(*[s.c for s in specs])
        res = (CglResult * len(specs))()
        if out is None:
            betas = np.empty((len(specs), self.p))
        else:
            betas = out
            if (betas.dtype != np.float64 or betas.shape != (len(specs), self.p)
                    or not betas.flags.c_contiguous or not betas.flags.writeable):
                raise ValueError(f"out must be a writeable C-contiguous float64 array of shape "
                                 f"{(len(specs), self.p)}")
        check(self.lib.cgl_solve_batch(self.h, arr, len(specs), _dptr(betas), res))
        return [_result(res[i], betas[i]) for i in range(len(specs))]

    def solve_batch_dual(self, specs: list[NodeSpec]):
        """solve_batch plus each bound's witness: returns (results, dual_betas), where row i of
        dual_betas is the iterate whose dual point -grad f(X beta) gave results[i].lower_bound
        (NaN rows for nodes that are not on the batched engine)."""
        arr = (CglNode * len(specs))(*[s.c for s in specs])
        res = (CglResult * len(specs))()
        betas = np.empty((len(specs), self.p))
        duals = np.empty((len(specs), self.p))
        check(self.lib.cgl_solve_batch_dual(self.h, arr, len(specs), _dptr(betas), res,
                                            _dptr(duals)))
        return [_result(res[i], betas[i]) for i in range(len(specs))], duals

    def certify(self, beta, Z0=(), Z1=()):
        spec = NodeSpec(self.p, Z0=Z0, Z1=Z1)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        P, D = C.c_double(), C.c_double()
        check(self.lib.cgl_certify(self.h, C.byref(spec.c), _dptr(b), C.byref(P), C.byref(D)))
        return P.value, D.value

    def matvec(self, v, trans=False):
        v = np.ascontiguousarray(v, dtype=np.float64)
        out = np.empty(self.p if trans else self.n)
        check(self.lib.cgl_problem_matvec(self.h, 1 if trans else 0, _dptr(v), _dptr(out)))
        return out


def node_validate(spec: NodeSpec, p: int, k: int) -> bool:
    """Host-side check of a node against (p, k) (cgl_node_validate; no device needed). Raises
    CglError for an invalid node; returns True when the node is infeasible (|Z1| > k)."""
    inf = C.c_int32()
    check(load().cgl_node_validate(C.byref(spec.c), int(p), int(k), C.byref(inf)))
    return bool(inf.value)


def prox_node_batch(ctx: Context, W, rho, M, k, sets=None):
    """Device prox for each row of W; sets: None or a list of (Z0, Z1). Returns (beta, g)."""
    W = np.ascontiguousarray(np.atleast_2d(W), dtype=np.float64)
    count, p = W.shape
    specs = [NodeSpec(p, Z0=z0, Z1=z1) for (z0, z1) in sets] if sets is not None else None
    arr = (CglNode * count)(*[s.c for s in specs]) if specs else None
    beta = np.empty_like(W)
    g = np.empty(count)
    check(ctx.lib.cgl_prox_node_batch(ctx.h, float(rho), float(M), int(k), arr, _dptr(W), count,
                                      p, _dptr(beta), _dptr(g)))
    return beta, g


def prox_batch_noalloc(ctx: Context, W, beta, g, rho, M, k):
    """cgl_prox_batch_noalloc on device buffers (objects with data_ptr() and shape): W and beta
    (count, p) float64, g None or (count,) float64. Enqueued on the context's stream; the caller
    synchronises that stream before reading the outputs."""
    count, p = (int(s) for s in W.shape)
    if tuple(beta.shape) != (count, p) or (g is not None and tuple(g.shape) != (count,)):
        raise ValueError("output shapes do not match W")
    check(ctx.lib.cgl_prox_batch_noalloc(ctx.h, float(rho), float(M), int(k),
                                         C.c_void_p(W.data_ptr()), count, p,
                                         C.c_void_p(beta.data_ptr()),
                                         C.c_void_p(g.data_ptr()) if g is not None else None))


class Server:
    """Continuous-batching request server over resident problems (cgl_server_*).

    submit() copies the node and returns a ticket; poll() runs one scheduling round and returns
    the finished requests as (ticket, Result with beta, latency seconds)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, max_slots: int = 256):
        self.ctx = ctx
        self.lib = ctx.lib
        self.h = C.c_void_p()
        check(self.lib.cgl_server_create(ctx.h, int(hbm_budget_bytes), int(max_slots),
                                          C.byref(self.h)))
        self._pmax = 0
        self._p = {}

    def submit(self, prob: "Problem", spec: NodeSpec) -> int:
        t = C.c_uint64()
        check(self.lib.cgl_server_submit(self.h, prob.h, C.byref(spec.c), C.byref(t)))
        self._pmax = max(self._pmax, prob.p)
        self._p[t.value] = prob.p
        return t.value

    def poll(self, max_results: int = 256):
        tickets = (C.c_uint64 * max_results)()
        res = (CglResult * max_results)()
        stride = max(self._pmax, 1)
        betas = np.empty((max_results, stride))
        lat = np.empty(max_results)
        got = C.c_int32()
        check(self.lib.cgl_server_poll(self.h, max_results, tickets, res, _dptr(betas), stride,
                                       _dptr(lat), C.byref(got)))
        out = []
        for i in range(got.value):
            t = int(tickets[i])
            p = self._p.pop(t, stride)
            out.append((t, _result(res[i], betas[i, :p].copy()), float(lat[i])))
        return out

    def cancel(self, ticket: int) -> None:
        check(self.lib.cgl_server_cancel(self.h, C.c_uint64(ticket)))

    def stats(self):
        q, r, d = C.c_int32(), C.c_int32(), C.c_int32()
        check(self.lib.cgl_server_stats(self.h, C.byref(q), C.byref(r), C.byref(d)))
        return {"queued": q.value, "running": r.value, "done": d.value}

    def close(self) -> None:
        if self.h:
            check(self.lib.cgl_server_destroy(self.h))
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

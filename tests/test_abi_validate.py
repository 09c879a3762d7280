"""Argument validation of the C ABI without a GPU: node specs through cgl_node_validate, and the
value checks of cgl_problem_create, which run before the context is looked at (a NULL context
with a bad argument reports the argument; with good arguments it reports the context)."""
import ctypes as C
import math
import os

import numpy as np
import pytest

from paper_2502_09502_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="library not built")


def _validate(p=20, k=4, **kw):
    spec = _lib.NodeSpec(p, **kw)
    return _lib.node_validate(spec, p, k)


def _err(fn):
    with pytest.raises(_lib.CglError) as e:
        fn()
    assert e.value.code == _lib.E_INVAL
    return str(e.value)


def test_valid_nodes_and_infeasibility():
    assert _validate() is False
    assert _validate(Z0=[0, 5, 19], Z1=[1, 2]) is False
    assert _validate(Z1=[1, 2, 3, 4]) is False          # |Z1| = k: k' = 0, still feasible
    assert _validate(Z1=[1, 2, 3, 4, 5]) is True        # |Z1| > k: infeasible, not an error
    assert _validate(Z0=np.arange(20)) is False         # everything fixed to zero
    assert _validate(warm_start=np.linspace(-3, 3, 20)) is False
    assert _validate(incumbent=12.5) is False


@pytest.mark.parametrize("kw, msg", [
    (dict(Z0=[20]), "fixed_zero index out of range"),
    (dict(Z0=[-1]), "fixed_zero index out of range"),
    (dict(Z1=[25]), "fixed_in index out of range"),
    (dict(Z0=[3, 3]), "duplicate fixed_zero"),
    (dict(Z1=[2, 2]), "duplicate fixed_in"),
    (dict(Z0=[7], Z1=[7]), "fixed both"),
    (dict(tol=-1e-6), "tol"),
    (dict(tol=math.nan), "tol"),
    (dict(max_iter=0), "max_iter"),
    (dict(check_every=0), "check_every"),
    (dict(precision=7), "precision"),
    (dict(incumbent=math.nan), "incumbent"),
    (dict(warm_start=np.r_[np.zeros(19), np.nan]), "warm start"),
    (dict(warm_start=np.r_[np.inf, np.zeros(19)]), "warm start"),
])
def test_invalid_nodes(kw, msg):
    assert msg in _err(lambda: _validate(**kw))


def test_null_and_negative_sizes():
    lib = _lib.load()
    n = _lib.CglNode()
    lib.cgl_node_init(C.byref(n))
    assert lib.cgl_node_validate(None, 10, 2, None) == _lib.E_INVAL
    assert lib.cgl_node_validate(C.byref(n), 0, 2, None) == _lib.E_INVAL
    assert lib.cgl_node_validate(C.byref(n), 10, 0, None) == _lib.E_INVAL
    n.n_zero = 3  # positive size with a NULL list
    assert lib.cgl_node_validate(C.byref(n), 10, 2, None) == _lib.E_INVAL
    assert b"NULL" in lib.cgl_last_error()
    n.n_zero = -1
    assert lib.cgl_node_validate(C.byref(n), 10, 2, None) == _lib.E_INVAL


def _create(X, y, loss="ls", lam2=1e-3, M=2.0, k=3, L=0.0, x_dtype=None, n=None, p=None,
            ldx=None):
    """cgl_problem_create with a NULL context; returns (status, message)."""
    lib = _lib.load()
    X = np.ascontiguousarray(X)
    dt = x_dtype if x_dtype is not None else {np.dtype(np.float64): _lib.F64,
                                              np.dtype(np.float32): _lib.F32,
                                              np.dtype(np.uint16): _lib.BF16}[X.dtype]
    nn, pp = X.shape
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = C.c_void_p()
    st = lib.cgl_problem_create(None, X.ctypes.data_as(C.c_void_p), dt, _lib.MEM_HOST,
                                nn if n is None else n, pp if p is None else p,
                                pp if ldx is None else ldx, _lib._dptr(y), _lib.LOSS[loss],
                                lam2, M, k, L, C.byref(out))
    assert not out.value
    return st, lib.cgl_last_error().decode()


def _data(n=30, p=8, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, p)), rng.standard_normal(n)


def test_problem_values_checked_before_context():
    X, y = _data()
    assert _create(X, y) == (_lib.E_INVAL, "ctx is NULL")
    ylab = np.where(y > 0, 1.0, -1.0)
    assert _create(X, ylab, loss="logistic") == (_lib.E_INVAL, "ctx is NULL")
    assert _create(X, np.abs(y), loss="poisson", L=5.0)[1] == "ctx is NULL"


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_X_rejected(dtype, bad):
    X, y = _data()
    X[7, 3] = bad
    X[0, 0] = bad
    if dtype == "f32":
        X = X.astype(np.float32)
    elif dtype == "bf16":
        X = (X.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    st, msg = _create(X, y)
    assert st == _lib.E_INVAL and "X has 2 non-finite entries" in msg


def test_padding_past_p_is_not_read_for_finiteness():
    # ldx > p: the columns past p are not part of X and may hold anything
    X, y = _data(p=10)
    X[:, 8:] = np.nan
    st, msg = _create(X, y, p=8, ldx=10)
    assert (st, msg) == (_lib.E_INVAL, "ctx is NULL")


@pytest.mark.parametrize("kw, msg", [
    (dict(lam2=0.0), "lambda2"),
    (dict(lam2=math.inf), "lambda2"),
    (dict(M=-1.0), "M must be"),
    (dict(M=math.nan), "M must be"),
    (dict(k=0), "k must be"),
    (dict(n=0), "n and p"),
    (dict(p=0), "n and p"),
    (dict(p=40000), "p > 32768"),
    (dict(ldx=5), "ldx < p"),
    (dict(x_dtype=9), "x_dtype"),
    (dict(loss="poisson"), "Lipschitz"),
])
def test_problem_argument_errors(kw, msg):
    X, y = _data()
    st, m = _create(X, y, **kw)
    assert st == _lib.E_INVAL and msg in m, m


@pytest.mark.parametrize("loss, y, msg", [
    ("ls", np.r_[np.ones(29), np.nan], "non-finite y"),
    ("logistic", np.r_[np.ones(29), 0.5], "labels must be -1 or +1"),
    ("sqhinge", np.r_[np.ones(29), 0.0], "labels must be -1 or +1"),
    ("poisson", np.r_[np.ones(29), -1.0], "Poisson responses"),
    ("gamma", np.r_[np.ones(29), 0.0], "Gamma responses"),
])
def test_response_range(loss, y, msg):
    X, _ = _data()
    st, m = _create(X, y, loss=loss, L=3.0)
    assert st == _lib.E_INVAL and msg in m, m


def test_null_handles_are_refused_without_a_device():
    lib = _lib.load()
    res = _lib.CglResult()
    n = _lib.CglNode()
    lib.cgl_node_init(C.byref(n))
    assert lib.cgl_solve_node(None, C.byref(n), None, C.byref(res)) == _lib.E_INVAL
    assert lib.cgl_solve_batch(None, C.byref(n), 1, None, C.byref(res)) == _lib.E_INVAL
    assert lib.cgl_solve_batch_dual(None, C.byref(n), 1, None, C.byref(res), None) == _lib.E_INVAL
    assert lib.cgl_certify(None, C.byref(n), None, None, None) == _lib.E_INVAL
    out = C.c_void_p()
    assert lib.cgl_server_create(None, 0, 16, C.byref(out)) == _lib.E_INVAL
    got = C.c_int32()
    assert lib.cgl_server_poll(None, 0, None, None, None, 0, None, C.byref(got)) == _lib.E_INVAL
    # destroying nothing is a no-op
    assert lib.cgl_problem_destroy(None) == _lib.OK
    assert lib.cgl_server_destroy(None) == _lib.OK
    assert lib.cgl_ctx_destroy(None) == _lib.OK

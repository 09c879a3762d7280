"""The allocation-free prox entry point (cgl_prox_batch_noalloc) against cgl_prox_node_batch on
the same inputs: two calls in a row through the C ABI, the second with fewer and shorter vectors
(the fixed scratch keeps the first call's contents), plus the size limits it rejects."""
import numpy as np
import pytest

import oracle
from paper_2502_09502_amd import _lib
from paper_2502_09502_amd.devmem import DeviceArray, Stream

pytestmark = pytest.mark.gpu


def _inputs(count, p, seed):
    rng = np.random.default_rng([seed, count, p])
    W = rng.standard_normal((count, p))
    W[0, : min(p, 5)] = 0.0                      # zeros (sgn 0)
    if count > 1:
        W[1, :] = np.round(W[1, :], 1)           # ties in |w|
    return W


def _noalloc(ctx, stream, W, rho, M, k):
    count, p = W.shape
    Wd = DeviceArray.from_numpy(W)
    Bd = DeviceArray((count, p), np.float64)
    Gd = DeviceArray((count,), np.float64)
    _lib.prox_batch_noalloc(ctx, Wd, Bd, Gd, rho, M, k)
    stream.synchronize()
    out = Bd.numpy(), Gd.numpy()
    for a in (Wd, Bd, Gd):
        a.free()
    return out


def test_noalloc_prox_matches_prox_node_batch_twice():
    stream = Stream(0)
    ctx = _lib.Context(0, stream.h)
    # first call: several tiles of the workgroup's per-thread slices and a ragged tail; second
    # call: fewer, shorter vectors and another k, after the first left its states in the scratch
    for count, p, rho, M, k, seed in ((96, 5003, 1.0, 1.0, 10, 1), (7, 300, 2.5, 0.7, 3, 2)):
        W = _inputs(count, p, seed)
        beta, g = _noalloc(ctx, stream, W, rho, M, k)
        ref_b, ref_g = _lib.prox_node_batch(ctx, W, rho, M, k)
        assert np.array_equal(beta, ref_b), np.max(np.abs(beta - ref_b))
        assert np.array_equal(g, ref_g)
        # and the oracle on two rows (prox of g/rho by Alg. 1 and the Moreau identity)
        for i in (0, count - 1):
            ob = oracle.prox_g(W[i], rho, M, k)
            assert np.max(np.abs(beta[i] - ob)) <= 1e-11 * max(1.0, np.max(np.abs(W[i])))
    ctx.close()
    stream.close()


def test_noalloc_prox_rejects_sizes_beyond_its_scratch():
    stream = Stream(0)
    ctx = _lib.Context(0, stream.h)
    W = DeviceArray((1, 8), np.float64)
    B = DeviceArray((1, 8), np.float64)
    lib = ctx.lib
    import ctypes as C
    for count, p in ((4097, 8), (1, 32769), (-1, 8), (1, 0)):
        rc = lib.cgl_prox_batch_noalloc(ctx.h, 1.0, 1.0, 3, C.c_void_p(W.data_ptr()), count, p,
                                        C.c_void_p(B.data_ptr()), None)
        assert rc == _lib.E_INVAL, (count, p)
    rc = lib.cgl_prox_batch_noalloc(ctx.h, 1.0, 1.0, 300, C.c_void_p(W.data_ptr()), 1, 8,
                                    C.c_void_p(B.data_ptr()), None)
    assert rc == _lib.OK  # k >= p: every coordinate in the budget
    stream.synchronize()
    W.free()
    B.free()
    ctx.close()
    stream.close()

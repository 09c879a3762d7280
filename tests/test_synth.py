"""The seeded generator follows the synthetic recipe of App. B.2 (with the readings stated in
``paper_2502_09502_amd.synth``)."""
import numpy as np

from paper_2502_09502_amd import synth


def test_beta_star_positions():
    assert list(np.nonzero(synth.beta_star(50, 5))[0]) == [9, 19, 29, 39, 49]
    assert np.count_nonzero(synth.beta_star(10000, 10)) == 10


def test_design_is_standardised_and_toeplitz_correlated():
    X = synth.design_matrix(20000, 6, np.random.default_rng(0))
    np.testing.assert_allclose(X.mean(axis=0), 0, atol=1e-12)
    np.testing.assert_allclose((X * X).sum(axis=0), 20000, rtol=1e-12)
    C = X.T @ X / 20000
    for lag in (1, 2, 3):
        assert abs(np.mean(np.diag(C, lag)) - 0.5 ** lag) < 0.02


def test_labels():
    d = synth.make_dataset(4000, 40, 4, loss="ls", config_id=90)
    resid = d.y - d.X @ d.beta_star
    u = d.X @ d.beta_star
    assert abs(np.var(resid) / (u @ u / d.n / 5.0) - 1) < 0.1  # SNR = 5
    dl = synth.make_dataset(4000, 40, 4, loss="logistic", config_id=90)
    assert set(np.unique(dl.y)) == {-1.0, 1.0}


def test_bf16_rounding_is_rne():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1.0 + 2 ** -9], dtype=np.float32)
    bits = synth.to_bf16_bits(x)
    assert list(bits) == [0x3F80, 0x3F80, 0x3F82, 0xC020, 0x3F80]
    np.testing.assert_array_equal(synth.bf16_bits_to_f32(bits)[[0, 3]], [1.0, -2.5])


def test_node_sets_disjoint_and_seeded():
    a = synth.node_sets(1000, 10, 50, 20)
    b = synth.node_sets(1000, 10, 50, 20)
    for (z0, z1), (w0, w1) in zip(a, b):
        assert np.array_equal(z0, w0) and np.array_equal(z1, w1)
        assert len(np.intersect1d(z0, z1)) == 0 and len(z0) <= 20 and len(z1) <= 10

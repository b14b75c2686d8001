"""Pins of the CPU reference network: reverse-mode gradient against central
finite differences of the FP64 loss, closed-form special cases, Adam step."""
import numpy as np

from oracle import mlp as M

LO = np.array([0.0, 0.0, 0.0])
HI = np.array([8.0, 2.0, 2.0])


def _batch(seed, n=37):
    rng = np.random.default_rng(seed)
    x = rng.uniform(LO, HI, (n, 3))
    sdf = rng.normal(0, 0.05, n)
    return x, sdf


def test_param_count():
    assert M.N_PARAMS == 64 * 64 + 64 + 2 * (64 * 64 + 64) + 64 + 1 == 12545


def test_features_closed_form():
    B = M.fourier_matrix(0, 1.0)
    phi = M.features(np.array([[4.0, 1.0, 1.0]]), LO, HI, B)  # box centre -> xh = 0
    np.testing.assert_allclose(phi[0, :32], 0.0, atol=1e-15)
    np.testing.assert_allclose(phi[0, 32:], 1.0)
    phi = M.features(np.array([[8.0, 2.0, 2.0]]), LO, HI, B)  # corner -> xh = 1
    z = 2 * np.pi * B.sum(1)
    np.testing.assert_allclose(phi[0], np.concatenate([np.sin(z), np.cos(z)]), rtol=1e-14)


def test_zero_weights_output_is_bias():
    p = M.unpack(np.zeros(M.N_PARAMS))
    p["b4"][0] = 0.3
    th = M.pack(p)
    x, _ = _batch(1)
    np.testing.assert_array_equal(M.forward(th, x, LO, HI, M.fourier_matrix(0, 1.0)), 0.3)


def test_gradient_matches_central_differences():
    th = M.init_params(3)
    B = M.fourier_matrix(3, 2.0)
    x, sdf = _batch(2)
    T = 0.1
    loss, g = M.loss_and_grad(th, x, sdf, LO, HI, B, T)
    assert abs(loss - M.loss_only(th, x, sdf, LO, HI, B, T)) < 1e-15
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(M.N_PARAMS, 120, replace=False), [M.N_PARAMS - 1]])
    for i in idx:
        h = 1e-6
        tp = th.copy(); tp[i] += h
        tm = th.copy(); tm[i] -= h
        fd = (M.loss_only(tp, x, sdf, LO, HI, B, T) - M.loss_only(tm, x, sdf, LO, HI, B, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_output_bias_gradient_closed_form():
    th = M.init_params(5)
    B = M.fourier_matrix(5, 1.0)
    x, sdf = _batch(4)
    _, g = M.loss_and_grad(th, x, sdf, LO, HI, B, 0.1)
    y = M.forward(th, x, LO, HI, B)
    assert abs(g[-1] - np.mean(y - np.clip(sdf, -0.1, 0.1))) < 1e-15


def test_adam_first_step_is_sign_step():
    th = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, -1e-3, 3.0])
    t1, m, v = M.adam_step(th, g, np.zeros(5), np.zeros(5), 1, 0.01)
    np.testing.assert_allclose(t1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)

"""Pins of the learned-propagator oracle (plain FP64 NumPy)."""
import numpy as np

import workloads as W
from oracle import learned as LR


def _rand_rho(rng, n, k):
    A = rng.normal(size=(k, n, n)) + 1j * rng.normal(size=(k, n, n))
    rho = A @ np.conj(np.swapaxes(A, 1, 2))
    return rho / np.trace(rho, axis1=1, axis2=2).real[:, None, None]


def test_encoding_round_trip_and_layout():
    rng = np.random.default_rng(0)
    rho = _rand_rho(rng, 5, 7)
    e = LR.encode(rho)
    assert e.shape == (7, 25)
    np.testing.assert_allclose(LR.decode(e, 5), rho, atol=1e-15)
    # diagonal first, then Re and Im of the upper triangle row-major
    assert e[0, 0] == rho[0, 0, 0].real and e[0, 5] == rho[0, 0, 1].real and e[0, 15] == rho[0, 0, 1].imag
    assert e[0, 14] == rho[0, 3, 4].real


def test_conditioning_of_the_five_level_family():
    c = LR.conditioning(W.vibronic(seed=100000))
    assert c.shape == (39,)
    assert set(np.unique(c[19:])) <= {0.0, 1.0}


def _tiny():
    rng = np.random.default_rng(1)
    window, n, n_cond = 3, 2, 2
    sizes = LR.layer_sizes(window, n * n, n_cond, 5, 3)
    params = LR.init_params(sizes, rng)
    params = [(W, rng.normal(size=b.shape) * 0.1) for W, b in params]
    X = rng.normal(size=(6, sizes[0]))
    Y = rng.normal(size=(6, n * n))
    return params, X, Y, n * n, window, sizes


def test_gradients_match_central_differences():
    params, X, Y, ne, window, sizes = _tiny()
    loss, grads = LR.loss_and_grads(params, X, Y, ne, window)
    flat = LR.flatten(params)
    gflat = LR.flatten(grads)
    rng = np.random.default_rng(2)
    for i in rng.choice(flat.size, 40, replace=False):
        h = 1e-6
        fp = flat.copy()
        fp[i] += h
        fm = flat.copy()
        fm[i] -= h
        lp, _ = LR.loss_and_grads(LR.unflatten(fp, sizes), X, Y, ne, window)
        lm, _ = LR.loss_and_grads(LR.unflatten(fm, sizes), X, Y, ne, window)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-8 + 1e-6 * abs(fd)


def test_first_adam_step_moves_by_lr_times_sign():
    params, X, Y, ne, window, sizes = _tiny()
    _, grads = LR.loss_and_grads(params, X, Y, ne, window)
    zeros = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    new, m, v = LR.adam_step(params, grads, zeros, zeros, 1, 1e-3)
    d = LR.flatten(new) - LR.flatten(params)
    g = LR.flatten(grads)
    big = np.abs(g) > 1e-4
    np.testing.assert_allclose(d[big], -1e-3 * np.sign(g[big]), rtol=1e-3)


def test_rollout_with_zero_output_layer_is_constant():
    rng = np.random.default_rng(3)
    n, window = 5, 4
    sizes = LR.layer_sizes(window, 25, 39, 8, 3)
    params = LR.init_params(sizes, rng)
    params[-1] = (np.zeros_like(params[-1][0]), np.zeros_like(params[-1][1]))
    rho = _rand_rho(rng, n, 3)
    init = np.repeat(LR.encode(rho)[:, None, :], window, axis=1)
    out = LR.rollout(params, init, rng.normal(size=(3, 39)), 5, n, window)
    np.testing.assert_allclose(out, np.repeat(LR.encode(rho)[:, None, :], 5, axis=1), atol=1e-14)


def test_trace_distance_of_pure_states():
    rng = np.random.default_rng(4)
    for _ in range(5):
        a = rng.normal(size=5) + 1j * rng.normal(size=5)
        b = rng.normal(size=5) + 1j * rng.normal(size=5)
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        t = LR.trace_distance(np.outer(a, a.conj()), np.outer(b, b.conj()))
        assert abs(t - np.sqrt(1 - abs(np.vdot(a, b)) ** 2)) < 1e-12

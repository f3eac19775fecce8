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


def test_gradients_with_propagated_residual_match_central_differences():
    params, X, Y, ne, window, sizes = _tiny()
    rng = np.random.default_rng(5)
    R = rng.normal(size=Y.shape)
    loss, grads = LR.loss_and_grads(params, X, Y, ne, window, R)
    flat, gflat = LR.flatten(params), LR.flatten(grads)
    for i in rng.choice(flat.size, 20, replace=False):
        h = 1e-6
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp, _ = LR.loss_and_grads(LR.unflatten(fp, sizes), X, Y, ne, window, R)
        lm, _ = LR.loss_and_grads(LR.unflatten(fm, sizes), X, Y, ne, window, R)
        assert abs((lp - lm) / (2 * h) - gflat[i]) <= 1e-8 + 1e-6 * abs(gflat[i])


def test_free_propagation_closed_form():
    """Diagonal H_S: rho_jk picks up exp(-i (E_j - E_k) dt); the trace and
    the spectrum are kept; U = 1 leaves rho unchanged."""
    rng = np.random.default_rng(6)
    n, dt = 5, 0.7
    E = rng.uniform(0, 0.3, n)
    U = LR.propagator({"h_el": np.diag(E)}, dt)
    rho = _rand_rho(rng, n, 4)
    got = LR.decode(LR.propagate(LR.encode(rho), U, n), n)
    ph = np.exp(-1j * (E[:, None] - E[None, :]) * dt)
    np.testing.assert_allclose(got, rho * ph, atol=1e-14)
    H = rng.normal(size=(n, n))
    U2 = LR.propagator({"h_el": (H + H.T) / 2}, dt)
    got2 = LR.decode(LR.propagate(LR.encode(rho), U2, n), n)
    np.testing.assert_allclose(np.trace(got2, axis1=1, axis2=2), 1.0, atol=1e-14)
    np.testing.assert_allclose(np.linalg.eigvalsh(got2), np.linalg.eigvalsh(rho), atol=1e-13)
    np.testing.assert_allclose(LR.propagate(LR.encode(rho), np.eye(n), n), LR.encode(rho), atol=1e-15)


def test_rollout_with_zero_network_is_free_propagation():
    rng = np.random.default_rng(7)
    n, window = 5, 3
    sizes = LR.layer_sizes(window, 25, 4, 6, 2)
    params = LR.init_params(sizes, rng)
    params[-1] = (np.zeros_like(params[-1][0]), np.zeros_like(params[-1][1]))
    H = rng.normal(size=(n, n))
    U = LR.propagator({"h_el": (H + H.T) / 2}, 0.3)
    rho = _rand_rho(rng, n, 2)
    init = np.repeat(LR.encode(rho)[:, None, :], window, axis=1)
    out = LR.rollout(params, init, rng.normal(size=(2, 4)), 4, n, window, np.stack([U, U]))
    ref = rho
    for k in range(4):
        ref = U @ ref @ np.conj(U.T)
        np.testing.assert_allclose(LR.decode(out[:, k], n), ref, atol=1e-13)


def test_skip_network_gradients_match_central_differences():
    rng = np.random.default_rng(9)
    window, n, nc = 2, 2, 3
    sizes = LR.layer_sizes(window, n * n, nc, 5, 2, skip=True)
    params = LR.init_params(sizes, rng, skip=True)
    params[-1] = (rng.normal(size=params[-1][0].shape) * 0.1, None)
    traj = rng.normal(size=(3, 6, n * n))
    cond = rng.normal(size=(3, nc))
    smp = np.array([[0, 2], [1, 3], [2, 4], [0, 1]])
    X, Y, R = LR.windows(traj, cond, smp, window, skip=True)
    assert X.shape[1] == sizes[0] == window * n * n + nc + nc * n * n
    # the bilinear block is cond (x) the last RDM
    np.testing.assert_allclose(X[1, window * n * n + nc:].reshape(nc, n * n), np.outer(cond[1], traj[1, 3]))
    loss, grads = LR.loss_and_grads(params, X, Y, n * n, window, R)
    flat, gflat = LR.flatten(params), LR.flatten(grads)
    assert flat.size == gflat.size
    for i in rng.choice(flat.size, 30, replace=False):
        h = 1e-6
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp, _ = LR.loss_and_grads(LR.unflatten(fp, sizes, True), X, Y, n * n, window, R)
        lm, _ = LR.loss_and_grads(LR.unflatten(fm, sizes, True), X, Y, n * n, window, R)
        assert abs((lp - lm) / (2 * h) - gflat[i]) <= 1e-8 + 1e-6 * abs(gflat[i])


def test_skip_only_network_is_linear_in_the_input():
    """Zero MLP output layer: the prediction is base + W_s x exactly."""
    rng = np.random.default_rng(10)
    sizes = LR.layer_sizes(2, 4, 3, 5, 2, skip=True)
    params = LR.init_params(sizes, rng, skip=True)
    params[-2] = (np.zeros_like(params[-2][0]), np.zeros_like(params[-2][1]))
    Ws = rng.normal(size=params[-1][0].shape)
    params[-1] = (Ws, None)
    X = rng.normal(size=(5, sizes[0]))
    pred, _ = LR.forward(params, X, 4, 2)
    np.testing.assert_allclose(pred, X[:, 4:8] + X @ Ws.T, atol=1e-13)

"""Pins for the oracle's guarded QR and Lanczos exponential."""
import math

import numpy as np
import scipy.linalg as sl

from oracle.ttns import completion_order, expv, qr_guarded


def _rand(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def test_full_rank_qr_is_householder_up_to_phase():
    rng = np.random.default_rng(1)
    A = _rand(rng, 37, 9)
    Q, R, g = qr_guarded(A, np.arange(37), 1e-8)
    assert g == 0
    Q0, R0 = np.linalg.qr(A)
    ph = np.diag(R0) / np.abs(np.diag(R0))
    np.testing.assert_allclose(Q, Q0 * ph[None, :], atol=1e-13)
    np.testing.assert_allclose(R, R0 / ph[:, None], atol=1e-12)
    assert np.all(np.diag(R).real > 0) and np.allclose(np.diag(R).imag, 0)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(9), atol=1e-14)
    assert np.allclose(np.tril(R, -1), 0)


def test_rank_deficient_completion_brute_force():
    rng = np.random.default_rng(2)
    rows, cols = 12, 6
    B = _rand(rng, rows, 2)
    A = B @ _rand(rng, 2, cols)            # rank 2
    A[:, 3] = 0.0
    order = np.arange(rows)[::-1]          # any order; here reversed
    Q, R, g = qr_guarded(A, order, 1e-8)
    assert g == cols - 2
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(cols), atol=1e-13)
    np.testing.assert_allclose(Q @ R, A, atol=1e-12)
    assert np.allclose(np.tril(R, -1), 0)
    # brute force: replay the completion rule by hand
    Qb = np.zeros_like(Q)
    k_data = 0
    for k in range(cols):
        if k in (0, 1):
            Qb[:, k] = Q[:, k]
            continue
        prev = Qb[:, :k]
        thr = 0.5 * (rows - k) / rows
        cand = next(i for i in order if 1 - np.sum(np.abs(prev[i]) ** 2) > thr)
        e = np.zeros(rows, complex)
        e[cand] = 1
        u = e - prev @ (prev.conj().T @ e)
        Qb[:, k] = u / np.linalg.norm(u)
    np.testing.assert_allclose(Q, Qb, atol=1e-12)


def test_completion_order_phys_fastest():
    # node axes (parent=2, phys=3, child=4); matricised towards the child
    order = completion_order((2, 3, 4), 2, 1)
    # rows are (parent, phys) row-major: row = p*3 + s; enumeration phys fastest
    assert list(order) == [0, 1, 2, 3, 4, 5]
    order = completion_order((2, 3, 4), 0, 1)
    # rows (phys, child) row-major: row = s*4 + c; phys fastest -> s varies first
    assert list(order[:4]) == [0, 4, 8, 1]


def test_expv_matches_expm():
    rng = np.random.default_rng(3)
    for n in (1, 5, 12, 40):
        X = _rand(rng, n, n)
        H = (X + X.conj().T) / 4
        x = _rand(rng, n)
        for z in (-0.05j, 0.3j, -1j):
            ref = sl.expm(z * H) @ x
            got = expv(lambda v: H @ v, x, z, 12)
            # exact once the Krylov space is the whole space; otherwise within
            # the a-priori bound 2 (|z||H|)^m / m! e^{|z||H|} (Taylor remainder)
            r = abs(z) * np.linalg.norm(H, 2)
            bound = 0.0 if n <= 12 else 2 * r ** 12 / math.factorial(12) * np.exp(r)
            assert np.linalg.norm(got - ref) <= (1e-12 + bound) * np.linalg.norm(x)


def test_expv_happy_breakdown_on_eigenvector():
    rng = np.random.default_rng(4)
    X = _rand(rng, 20, 20)
    H = X + X.conj().T
    w, U = np.linalg.eigh(H)
    info = {}
    got = expv(lambda v: H @ v, U[:, 3] * 2.0, -0.7j, 12, info=info)
    np.testing.assert_allclose(got, 2.0 * np.exp(-0.7j * w[3]) * U[:, 3], atol=1e-12)
    assert info.get("breakdown", 0) == 1

"""Pins of the energy-surface oracle (Eqs. 3-4: the effective Hamiltonian and
effective potential between bath Schmidt states and electronic states).

* Product initial state: one bath state (the vacuum), so the surfaces of H
  are the eigenvalues of H_S, and those of H - T are shifted by the chains'
  zero-point kinetic energy sum_n eps_n / 4 (<0|p^2|0> = 1/2).
* Exact references on a tree with full bond dimensions: the full state from
  expm, its SVD across electronic x environment, and the dense H and a dense
  kinetic energy built from the normal modes of each chain (eigenvectors of
  its tridiagonal matrix), not from the chain-site momenta the oracle's
  operator sum uses.
* The energy <psi|H|psi> equals c^H H^eff c for the Schmidt coefficients c
  (the state lies in the span), and the matrix is Hermitian.
"""
import numpy as np
import scipy.linalg as sl

import workloads as W
from oracle import ed
from oracle import surfaces as S
from oracle.chain import ohmic_chain
from oracle.model import boson_ops, build_tree, momentum_op
from oracle.ttns import TTNS


def test_product_state_surfaces_are_the_system_levels():
    m = W.vibronic_small(steps=1)
    tt = TTNS(build_tree(m))
    np.testing.assert_allclose(S.energy_surfaces(tt), np.linalg.eigvalsh(m["h_el"]), atol=1e-14)
    tv = TTNS(build_tree(m, potential=True))
    zp = sum(np.sum(ohmic_chain(c["alpha"], c["wc"], c["s"], c["L"])[1]) / 4 for c in m["chains"])
    np.testing.assert_allclose(S.energy_surfaces(tv), np.linalg.eigvalsh(m["h_el"]) - zp, atol=1e-13)


def _dense_kinetic(tree, model):
    """sum over every chain's normal modes of (w/2) P^2, P = sum_n U_nk p_n."""
    phys = tree.phys
    N = int(np.prod(phys))
    T = np.zeros((N, N), dtype=np.complex128)
    for c, ch in enumerate(model["chains"]):
        _, eps, hop = ohmic_chain(ch["alpha"], ch["wc"], ch["s"], ch["L"])
        M = np.diag(eps) + np.diag(hop, 1) + np.diag(hop, -1)
        w, U = np.linalg.eigh(M)
        nodes = tree.chain_nodes[c]
        p = momentum_op(ch["d"])
        pn = [ed.place({v: p}, phys) for v in nodes]
        for k in range(len(w)):
            P = sum(U[n, k] * pn[n] for n in range(len(nodes)))
            T += 0.5 * w[k] * (P @ P)
    return T


def _exact_surfaces(psi, Hd, n):
    M = psi.reshape(n, -1)
    _, s, Vh = np.linalg.svd(M, full_matrices=False)
    r = int(np.sum(s > 1e-8 * s[0]))
    B = []
    for i in range(r):
        for j in range(n):
            X = np.zeros((n, M.shape[1]), dtype=np.complex128)
            X[j] = Vh[i]
            B.append(X.reshape(-1))
    B = np.array(B).T
    return np.linalg.eigvalsh(B.conj().T @ Hd @ B), r


def test_surfaces_match_exact_evolution_with_full_bond_dimensions():
    m = W.vibronic(seed=9, n_levels=3, n_chains=2, L=2, d=3, D=100, steps=4)
    tree = build_tree(m)
    H = ed.dense_hamiltonian(tree)
    Tk = _dense_kinetic(tree, m)
    psi = sl.expm(-1j * H * m["dt"] * 4) @ ed.initial_full_state(tree)
    tt = TTNS(tree, rank_tol=1e-14)
    for _ in range(4):
        tt.step(m["dt"])
    ref_h, r = _exact_surfaces(psi, H, 3)
    assert r == 3
    np.testing.assert_allclose(S.energy_surfaces(tt), ref_h, atol=1e-9)
    tv = TTNS(build_tree(m, potential=True), rank_tol=1e-14)
    S.copy_state(tv, tt)
    ref_v, _ = _exact_surfaces(psi, H - Tk, 3)
    np.testing.assert_allclose(S.energy_surfaces(tv), ref_v, atol=1e-9)


def test_energy_lies_in_the_bath_subspace():
    m = W.vibronic_small(steps=3)
    tt = TTNS(build_tree(m))
    for _ in range(3):
        tt.step(m["dt"])
    Hm, s = S.effective_matrix(tt)
    assert np.abs(Hm - Hm.conj().T).max() < 1e-13
    C = tt.T[0]
    n = C.shape[0]
    U, ss, _ = np.linalg.svd(C.reshape(n, -1), full_matrices=False)
    c = np.array([U[j, i] * ss[i] for i in range(len(s)) for j in range(n)])
    assert abs((c.conj() @ Hm @ c).real - tt.energy()) < 1e-12

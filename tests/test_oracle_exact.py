"""Pins of the oracle against exact diagonalisation on tiny trees.

* With full bond dimensions the TTNS manifold is the whole Hilbert space, and
  the projector-splitting integrator is then exact for any step size
  (Lubich, Oseledets & Vandereycken, SINUM 2015): the oracle must reproduce
  expm(-i H t) psi0.
* H_eff at any node and H_bond on any edge must equal P^H H P for the
  embedding P defined by the current isometries.
* Root observables must equal the full-state expectation values.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W
from oracle import ed
from oracle.model import boson_ops, build_tree
from oracle.ttns import TTNS

TREES = {
    "spin+3 sites d3": lambda: W.spin_boson(L=3, d=3, D=100, delta=0.7, alpha=0.2, dt=0.1),
    "3 levels + 2x2 sites d3": lambda: W.vibronic(seed=5, n_levels=3, n_chains=2, L=2, d=3, D=100),
    "5 levels + 2x2 sites d3": lambda: W.vibronic(seed=6, n_levels=5, n_chains=2, L=2, d=3, D=100),
    "ER: 2 levels + 4x1 sites d2": lambda: dict(W.vibronic(seed=7, n_levels=2, n_chains=4, L=1, d=2, D=100),
                                                topology="er", er_D=100),
    # optimised boson basis: every site a node without physical leg plus a
    # basis node holding its Fock states (full basis: exact manifold)
    "OBB: spin + 3 sites d3": lambda: W.with_obb(W.spin_boson(L=3, d=3, D=100, delta=0.7, alpha=0.2, dt=0.1), 3),
    "OBB: 3 levels + 2x2 sites d2": lambda: W.with_obb(W.vibronic(seed=8, n_levels=3, n_chains=2, L=2, d=2,
                                                                  D=100), 2),
}


@pytest.mark.parametrize("name", list(TREES))
def test_full_bond_dims_reproduce_exact_evolution(name):
    m = TREES[name]()
    tree = build_tree(m)
    H = ed.dense_hamiltonian(tree)
    psi0 = ed.initial_full_state(tree)
    dt, n = m["dt"], 6
    for rank_tol, tol in ((1e-14, 1e-10), (1e-8, 1e-7)):
        t = TTNS(tree, rank_tol=rank_tol)
        assert np.allclose(t.full_state(), psi0)
        for _ in range(n):
            t.step(dt)
        ref = sl.expm(-1j * H * dt * n) @ psi0
        assert np.abs(t.full_state() - ref).max() < tol, (name, rank_tol)


@pytest.mark.parametrize("name", list(TREES))
def test_effective_hamiltonians_are_projections(name):
    m = TREES[name]()
    tree = build_tree(m)
    H = ed.dense_hamiltonian(tree)
    t = TTNS(tree, rank_tol=1e-14)
    for _ in range(2):
        t.step(m["dt"])
    rng = np.random.default_rng(0)
    for target in range(t.n):
        t.move_to(target)
        P = ed.embedding_node(t, target)
        X = rng.normal(size=t.shape[target]) + 1j * rng.normal(size=t.shape[target])
        ref = (P.conj().T @ H @ P) @ X.reshape(-1)
        got = t.apply_heff(target, X).reshape(-1)
        assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
        for u in t.nbrs[target]:
            # bond between target (made an isometry towards u) and u
            saved = [x.copy() for x in t.T], dict(t.env), t.centre
            R = t.qr_to(target, u)
            Pb = ed.embedding_bond(t, target, u)
            Rr = rng.normal(size=R.shape) + 1j * rng.normal(size=R.shape)
            ref = (Pb.conj().T @ H @ Pb) @ Rr.reshape(-1)
            got = t.apply_hbond(target, u, Rr).reshape(-1)
            assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
            t.T, t.env, t.centre = saved
    t.move_to(0)


@pytest.mark.parametrize("name", list(TREES))
def test_observables_match_full_state(name):
    m = TREES[name]()
    tree = build_tree(m)
    H = ed.dense_hamiltonian(tree)
    t = TTNS(tree)
    for _ in range(3):
        t.step(m["dt"])
    psi = t.full_state()
    n_el = tree.phys[0]
    M = psi.reshape(n_el, -1)
    np.testing.assert_allclose(t.rdm(), M @ M.conj().T, atol=1e-13)
    assert abs(t.norm2() - np.vdot(psi, psi).real) < 1e-13
    assert abs(t.energy() - np.vdot(psi, H @ psi).real) < 1e-12
    for i, h in enumerate(tree.heads):
        num = boson_ops(tree.phys[h])[2]
        ref = np.vdot(psi, ed.place({h: num}, tree.phys) @ psi).real
        assert abs(t.local_expectation(h, num).real - ref) < 1e-13


def test_paper_root_tensor_memory_model():
    """Fig. 2 / Methods: a star root carrying 7 chain bonds is an order-8
    tensor of 57 TB; with 5 electronic states and D = 50 on every chain bond
    in complex128 the shape logic gives 5 * 50^7 * 16 bytes = 56.8 TiB."""
    from oracle.ttns import clamp_bond_dims
    parent = [-1] + [0] * 7 + list(range(1, 8))
    phys = [5] + [100] * 14
    children = [[] for _ in parent]
    for v in range(1, len(parent)):
        children[parent[v]].append(v)
    D = clamp_bond_dims(parent, phys, [0] + [50] * 14, children)
    root_bytes = phys[0] * np.prod([D[c] for c in children[0]]) * 16
    assert abs(root_bytes / 2 ** 40 - 56.84) < 0.01


def _subtree(tree, v):
    out, stack = [], [v]
    while stack:
        u = stack.pop()
        out.append(u)
        stack.extend(c for c in range(len(tree.parent)) if tree.parent[c] == u)
    return sorted(out)


@pytest.mark.parametrize("name", list(TREES))
def test_bond_entropy_matches_full_state_schmidt_values(name):
    """Entanglement entropy across every bond against the Schmidt
    decomposition of the full state (subtree legs | the rest); zero for the
    product initial state."""
    m = TREES[name]()
    tree = build_tree(m)
    t = TTNS(tree)
    n = len(tree.parent)
    for v in range(1, n):
        assert abs(t.bond_entropy(v)) < 1e-12
    t.move_to(0)
    for _ in range(3):
        t.step(m["dt"])
    psi = t.full_state()
    dims = [tree.phys[u] for u in range(n)]
    for v in range(1, n):
        sub = _subtree(tree, v)
        assert sub == list(range(v, v + len(sub)))  # pre-order: contiguous legs
        X = psi.reshape(dims)
        rest = [u for u in range(n) if u not in sub]
        M = np.transpose(X, sub + rest).reshape(int(np.prod([dims[u] for u in sub])), -1)
        s = np.linalg.svd(M, compute_uv=False)
        p = s ** 2 / np.sum(s ** 2)
        p = p[p > 1e-300]
        ref = float(-np.sum(p * np.log(p)))
        t.move_to(0)
        assert abs(t.bond_entropy(v) - ref) < 1e-10, (name, v)

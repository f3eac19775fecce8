"""Physics pins of the oracle: closed forms, invariants and symmetries."""
import numpy as np
import scipy.linalg as sl

import workloads as W
from oracle.model import build_tree
from oracle.ttns import TTNS, run
from tests.pins import chain_displacement, dephasing_gamma, ohmic_J, stieltjes_chain


def test_norm_and_energy_conserved_with_truncated_bonds():
    m = W.spin_boson(D=4, steps=40, delta=0.6, alpha=0.2)
    _, h = run(m)
    assert np.abs(h["norm"] - 1.0).max() < 1e-10
    assert np.abs(h["energy"] - h["energy"][0]).max() < 1e-10
    m = W.vibronic_small(steps=3)
    _, h = run(m)
    assert np.abs(h["norm"] - 1.0).max() < 1e-10
    assert np.abs(h["energy"] - h["energy"][0]).max() < 1e-10


def test_pure_dephasing_matches_continuum_closed_form():
    """Delta = 0, psi0 = (|up> + |down>)/sqrt2: <sx>(t) = exp(-Gamma(t)) with
    Gamma = 8 alpha Cin(wc t) for J = 2 pi alpha w theta(wc - w) and the
    coupling sz (x) c0 (b0 + b0^+); the 10-site chain is reflection free
    over t <= 5 and the state has Schmidt rank 2 on every bond."""
    m = W.spin_boson(delta=0.0, init=(2 ** -0.5, 2 ** -0.5), steps=100)
    _, h = run(m)
    t = np.arange(101) * m["dt"]
    sx = 2 * h["rdm"][:, 0, 1].real
    assert np.abs(sx - np.exp(-dephasing_gamma(0.1, 1.0, t))).max() < 1e-6
    # populations stay at 1/2, the coherence stays real
    assert np.abs(h["rdm"][:, 0, 0].real - 0.5).max() < 1e-12
    assert np.abs(h["rdm"][:, 0, 1].imag).max() < 1e-10


def test_pure_dephasing_with_optimised_boson_basis():
    """The pure-dephasing state keeps every site in one of two coherent
    states (one per spin branch), a site basis of two states and bond
    dimension 2 would hold it.  With a three-state optimised boson basis and
    D = 3 (room for the one-site integrator's tangent directions) the tree
    (sites without physical legs, Fock states on the basis nodes, coupling
    and hopping acting there) follows the continuum's exp(-Gamma(t)) to the
    chain's own accuracy (the plain 10-site chain is 4e-7 off); with two
    basis states the splitting error (1.7e-5 at dt = 0.05, quartered at
    dt / 2) remains."""
    m = W.with_obb(W.spin_boson(delta=0.0, init=(2 ** -0.5, 2 ** -0.5), steps=100, D=3), 3)
    tt, h = run(m)
    assert tt.n == 1 + 2 * 10 and max(tt.D) <= 3
    t = np.arange(101) * m["dt"]
    sx = 2 * h["rdm"][:, 0, 1].real
    assert np.abs(sx - np.exp(-dephasing_gamma(0.1, 1.0, t))).max() < 2e-6
    assert np.abs(h["rdm"][:, 0, 0].real - 0.5).max() < 1e-12


def test_decoupled_spin_rabi():
    m = W.spin_boson(alpha=0.0, delta=0.7, D=4, L=4, d=4, steps=30, dt=0.1)
    _, h = run(m)
    t = np.arange(31) * 0.1
    sz = (h["rdm"][:, 0, 0] - h["rdm"][:, 1, 1]).real
    assert np.abs(sz - np.cos(0.7 * t)).max() < 1e-12


def test_decoupled_levels_follow_system_hamiltonian():
    m = W.vibronic(seed=11, n_chains=2, L=3, d=3, D=3, steps=5, alpha_range=(0.0, 0.0))
    _, h = run(m)
    rho0 = np.outer(m["init_el"], m["init_el"].conj())
    for k in range(6):
        U = sl.expm(-1j * m["h_el"] * m["dt"] * k)
        np.testing.assert_allclose(h["rdm"][k], U @ rho0 @ U.conj().T, atol=1e-12)


def test_independent_boson_multilevel_decoherence():
    """Diagonal H_S, 0/1 diagonal couplings: populations are constant and
    |rho_jk(t)| = |rho_jk(0)| prod_i exp(-(m_ij - m_ik)^2 Phi_i(t)),
    Phi_i = |c0 M^-1 (1 - e^{-iMt}) e0|^2 / 2 for chain i (coefficients from
    the independent Stieltjes procedure)."""
    m = W.vibronic(seed=12, n_levels=3, n_chains=2, L=6, d=6, D=4, steps=8)
    n = 3
    m["h_el"] = np.diag(np.diag(m["h_el"]))
    m["init_el"] = np.ones(n, dtype=np.complex128) / np.sqrt(n)
    _, h = run(m)
    t = np.arange(9) * m["dt"]
    masks = [np.diag(c["coupling"]).real for c in m["chains"]]
    phis = []
    for c in m["chains"]:
        c0, e, hop = stieltjes_chain(ohmic_J(c["alpha"], c["wc"]), c["wc"], c["L"])
        phis.append(0.5 * chain_displacement(c0, e, hop, t))
    for j in range(n):
        assert np.abs(h["rdm"][:, j, j].real - 1.0 / n).max() < 1e-10
        for k in range(n):
            expo = sum((mk[j] - mk[k]) ** 2 * ph for mk, ph in zip(masks, phis))
            np.testing.assert_allclose(np.abs(h["rdm"][:, j, k]), np.exp(-expo) / n, atol=2e-6)


def test_time_reversal():
    """The second-order step is symmetric: step(dt) then step(-dt) is the
    identity (after the bonds have filled, so no completion events)."""
    m = W.spin_boson(L=4, d=4, D=3, delta=0.5, alpha=0.3, dt=0.1)
    t = TTNS(build_tree(m))
    for _ in range(15):
        t.step(0.1)
    psi = t.full_state()
    g0 = t.stats["guarded"]
    t.step(0.1)
    t.step(-0.1)
    assert t.stats["guarded"] == g0
    assert np.abs(t.full_state() - psi).max() < 1e-10


def test_second_order_convergence():
    m = W.spin_boson(L=4, d=4, D=2, delta=0.5, alpha=0.3)
    T = 0.8

    def final(dt):
        t = TTNS(build_tree(m), rank_tol=1e-8)
        for _ in range(int(round(T / dt))):
            t.step(dt)
        return t.full_state()

    ref = final(0.0125)
    e1 = np.linalg.norm(final(0.2) - ref)
    e2 = np.linalg.norm(final(0.1) - ref)
    assert 3.0 < e1 / e2 < 5.0

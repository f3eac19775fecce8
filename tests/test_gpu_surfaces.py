"""GPU energy surfaces (Eqs. 3-4) against the oracle's.

The surfaces are the eigenvalues of the effective Hamiltonian (operator H)
and of the effective potential (operator H - T, a context built with
``potential`` that takes the state by ttns_copy_state) between the bath
Schmidt states of the root and the electronic states.  Bath states are kept
while s_i > rank_tol s_0 on both sides (the same rule), and both sides must
keep the same number.  Bars on the eigenvalues (energies of order
0.1-1 eV): a bath state of Schmidt value s is the state's component along
it divided by s, so the ~1e-13 difference of the two trajectories reaches
the surfaces amplified by up to s_0 / s_min: 1e-10 absolute with
rank_tol = 1e-3 (only well-determined bath states), 1e-8 with 1e-5 (all five
bath states of these trees, the smallest near 1.3e-5 s_0).
"""
import numpy as np
import pytest

import workloads as W
from oracle import surfaces as S
from oracle.chain import ohmic_chain
from oracle.model import build_tree
from oracle.ttns import TTNS

pytestmark = pytest.mark.gpu


def _T():
    from paper_1710_01362_amd import ttns as T
    return T


def _gpu_surfaces(m, steps, rank_tol, **opts):
    T = _T()
    h = T.Context([m], opts=T.default_opts(record_capacity=steps + 1, **opts))
    if steps:
        h.ttns_tdvp_step(m["dt"], steps)
    tes = h.energy_surfaces(0, rank_tol)
    v = T.Context([dict(m, potential=True)], opts=T.default_opts(record_capacity=2, **opts))
    v.copy_state_from(h)
    pes = v.energy_surfaces(0, rank_tol)
    h.close()
    v.close()
    return tes, pes


def _oracle_surfaces(m, steps, rank_tol):
    tt = TTNS(build_tree(m))
    for _ in range(steps):
        tt.step(m["dt"])
    tv = TTNS(build_tree(m, potential=True))
    S.copy_state(tv, tt)
    return S.energy_surfaces(tt, rank_tol), S.energy_surfaces(tv, rank_tol)


def test_product_state_surfaces_are_the_system_levels():
    m = W.vibronic_small(steps=1)
    tes, pes = _gpu_surfaces(m, 0, 1e-5)
    levels = np.linalg.eigvalsh(m["h_el"])
    zp = sum(np.sum(ohmic_chain(c["alpha"], c["wc"], c["s"], c["L"])[1]) / 4 for c in m["chains"])
    np.testing.assert_allclose(tes, levels, atol=1e-12)
    np.testing.assert_allclose(pes, levels - zp, atol=1e-12)


@pytest.mark.parametrize("rank_tol,tol", [(1e-3, 1e-10), (1e-5, 1e-8)])
@pytest.mark.parametrize("kind", ["star", "er", "obb"])
def test_surfaces_after_evolution_match_oracle(kind, rank_tol, tol):
    m = W.vibronic_small(steps=4)
    if kind == "er":
        m = dict(m, topology="er")
    elif kind == "obb":
        m = W.with_obb(W.vibronic_small(steps=4, L=4, d=8, D=4), 3)
    tes, pes = _gpu_surfaces(m, 4, rank_tol)
    ot, op = _oracle_surfaces(m, 4, rank_tol)
    assert len(tes) == len(ot) and len(pes) == len(op) and len(tes) > 5
    assert np.abs(tes - ot).max() <= tol, np.abs(tes - ot).max()
    assert np.abs(pes - op).max() <= tol, np.abs(pes - op).max()


def test_surfaces_of_the_five_level_tree_root():
    """Full-size root (5 x 20^4 on the matrix cores) after two steps."""
    m = W.vibronic_reference()
    tes, pes = _gpu_surfaces(m, 2, 1e-3)
    ot, op = _oracle_surfaces(m, 2, 1e-3)
    assert len(tes) == len(ot)
    assert np.abs(tes - ot).max() <= 1e-10, np.abs(tes - ot).max()
    assert np.abs(pes - op).max() <= 1e-10, np.abs(pes - op).max()
    print("five-level tree after 2 steps: %d bath states, lowest surfaces %s" % (len(tes) // 5, tes[:5]))

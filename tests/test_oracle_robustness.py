"""Parity stability of the rank-guarded QR (the reading of rank-deficient
centres: a column whose residual is below rank_tol |A|_F is completed by a
fixed unit-vector rule).

The product initial state makes most QR inputs rank deficient, so the
columns that span a node's tangent directions are chosen by that rule, not
by rounding.  If the rule is stable, a perturbation of the initial state far
below the guard (1e-14 against 1e-8) changes the trajectory only at the size
of the perturbation amplified by the dynamics, never by an O(1) change of a
completed column: the populations move by at most 1e-7.
"""
import numpy as np

import workloads as W
from oracle.model import build_tree
from oracle.ttns import TTNS


def _populations(model, steps, noise, seed=5):
    tt = TTNS(build_tree(model), krylov=model.get("krylov", 12))
    if noise:
        rng = np.random.default_rng(seed)
        C = tt.T[0]
        tt.T[0] = C + noise * (rng.normal(size=C.shape) + 1j * rng.normal(size=C.shape))
        tt.T[0] /= np.linalg.norm(tt.T[0])
        # the environments towards the root do not depend on the root tensor
    pops = [np.diag(tt.rdm()).real.copy()]
    for _ in range(steps):
        tt.step(model["dt"])
        pops.append(np.diag(tt.rdm()).real.copy())
    return np.array(pops), tt.stats["guarded"]


def test_spin_boson_trajectory_stable_under_tiny_perturbation():
    m = W.spin_boson_reference()
    p0, g0 = _populations(m, 120, 0.0)
    p1, g1 = _populations(m, 120, 1e-14)
    assert g0 > 0  # the guard is exercised
    assert np.abs(p1 - p0).max() <= 1e-7


def test_five_level_tree_stable_under_tiny_perturbation():
    m = W.vibronic_small(steps=30)
    p0, g0 = _populations(m, 30, 0.0)
    p1, g1 = _populations(m, 30, 1e-14)
    assert g0 > 0
    assert np.abs(p1 - p0).max() <= 1e-7


def test_guard_threshold_separates_perturbation_from_rank():
    """A perturbation above the guard (1e-6) is a real change of rank: the
    completion is then replaced by the perturbed direction and the number
    of guarded columns drops."""
    m = W.vibronic_small(steps=3)
    _, g0 = _populations(m, 3, 0.0)
    _, g1 = _populations(m, 3, 1e-6)
    assert g1 < g0

"""Pin: closed-form chain coefficients vs the numerical Stieltjes procedure."""
import numpy as np
import pytest

from oracle.chain import ohmic_chain
from tests.pins import ohmic_J, stieltjes_chain


@pytest.mark.parametrize("alpha,wc,s,L", [(0.1, 1.0, 1.0, 10), (0.17, 0.2, 1.0, 40), (0.3, 2.0, 0.5, 12)])
def test_closed_form_matches_stieltjes(alpha, wc, s, L):
    c0, eps, t = ohmic_chain(alpha, wc, s, L)
    c0_r, eps_r, t_r = stieltjes_chain(ohmic_J(alpha, wc, s), wc, L)
    tol = 1e-12 if s == 1.0 else 1e-9
    assert abs(c0 - c0_r) <= tol * wc
    np.testing.assert_allclose(eps, eps_r, atol=tol * wc, rtol=0)
    np.testing.assert_allclose(t, t_r, atol=tol * wc, rtol=0)


def test_reference_spin_boson_coefficients_shape():
    c0, eps, t = ohmic_chain(0.1, 1.0, 1.0, 10)
    assert eps.shape == (10,) and t.shape == (9,)
    # alpha = 0.1, wc = 1, s = 1: c0 = sqrt(2 alpha / (1 + s)) wc
    assert abs(c0 - np.sqrt(0.1)) < 1e-15
    # semi-infinite chain limit: eps_n -> wc/2, t_n -> wc/4
    c0, eps, t = ohmic_chain(0.1, 1.0, 1.0, 2000)
    assert abs(eps[-1] - 0.5) < 1e-6 and abs(t[-1] - 0.25) < 1e-6

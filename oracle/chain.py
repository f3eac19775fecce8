"""Chain mapping of a bosonic environment (test infrastructure, CPU oracle).

The paper maps each cluster of vibrational modes onto a semi-infinite chain
with the orthogonal-polynomial transformation (section "Interface to TTNS",
citing Chin et al., J. Math. Phys. 51, 092109 (2010)).  For the power-law
spectral density with a hard cutoff,

    J(w) = 2 pi alpha wc (w / wc)^s  theta(wc - w),

the recurrence coefficients of the associated (shifted Jacobi) polynomials are
known in closed form; this module writes them out.  The chain Hamiltonian is

    H_chain = sum_n eps_n b_n^+ b_n + sum_n t_n (b_n^+ b_{n+1} + h.c.),

and the system couples to site 0 through c0 (b_0 + b_0^+), with
c0 = sqrt(eta0 / pi) and eta0 = integral of J over [0, wc].
"""
import numpy as np


def ohmic_chain(alpha, wc, s, L):
    """Return (c0, eps[L], t[L-1]) for the hard-cutoff power-law density."""
    alpha = float(alpha)
    wc = float(wc)
    s = float(s)
    eta0 = 2.0 * np.pi * alpha * wc * wc / (1.0 + s)
    c0 = np.sqrt(eta0 / np.pi)
    n = np.arange(L, dtype=np.float64)
    eps = 0.5 * wc * (1.0 + s * s / ((s + 2 * n) * (s + 2 * n + 2)))
    m = np.arange(max(L - 1, 0), dtype=np.float64)
    t = (wc * (m + 1) * (m + 1 + s) / ((s + 2 * m + 2) * (s + 2 * m + 3))
         * np.sqrt((s + 2 * m + 3) / (s + 2 * m + 1)))
    return c0, eps, t

"""Independent references for the oracle pins (no import from oracle/).

* ``stieltjes_chain``: chain coefficients of a spectral density by the
  discretised Stieltjes (Lanczos) procedure on Gauss-Legendre nodes -- the
  orthogonal-polynomial recurrence computed numerically, not from the closed
  form.
* ``dephasing_gamma``: decoherence exponent of the pure-dephasing spin-boson
  model in the continuum, Gamma(t) = (8/pi) int J(w) sin^2(wt/2)/w^2 dw,
  which for the Ohmic hard-cutoff density is 8 alpha Cin(wc t).
* ``chain_displacement``: the same exponent for a finite chain from the
  single-particle propagator, |c0 M^-1 (1 - e^{-iMt}) e0|^2.
"""
import numpy as np
import scipy.linalg as sl
from scipy.special import sici


def stieltjes_chain(J, wc, L, nquad=4000):
    x, g = np.polynomial.legendre.leggauss(nquad)
    w = 0.5 * wc * (x + 1.0)
    wt = 0.5 * wc * g * J(w)
    eta0 = wt.sum()
    q = np.sqrt(wt / eta0)
    Q = [q]
    a, b = [], []
    prev = np.zeros_like(q)
    beta = 0.0
    for n in range(L):
        v = w * Q[-1] - beta * prev
        alpha = np.dot(Q[-1], v)
        v = v - alpha * Q[-1]
        for qq in Q:  # full reorthogonalisation
            v = v - np.dot(qq, v) * qq
        a.append(alpha)
        beta = np.linalg.norm(v)
        b.append(beta)
        prev = Q[-1]
        Q.append(v / beta)
    return np.sqrt(eta0 / np.pi), np.array(a), np.array(b[:L - 1])


def ohmic_J(alpha, wc, s=1.0):
    return lambda w: 2 * np.pi * alpha * wc * (w / wc) ** s * (w <= wc)


def cin(x):
    si, ci = sici(x)
    return np.euler_gamma + np.log(x) - ci


def dephasing_gamma(alpha, wc, t):
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    pos = t > 0
    out[pos] = 8.0 * alpha * cin(wc * t[pos])
    return out


def chain_displacement(c0, eps, hop, t):
    M = np.diag(eps) + np.diag(hop, 1) + np.diag(hop, -1)
    e0 = np.zeros(len(eps))
    e0[0] = 1.0
    Minv = np.linalg.inv(M)
    out = []
    for tt in np.atleast_1d(t):
        v = c0 * Minv @ ((np.eye(len(eps)) - sl.expm(-1j * M * tt)) @ e0)
        out.append(np.vdot(v, v).real)
    return np.array(out)

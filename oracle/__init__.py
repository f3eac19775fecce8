"""CPU oracle for the TTNS one-site TDVP hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex128 NumPy
implementation of what the HIP library computes: the orthogonal-polynomial
chain mapping of the bosonic environments, the star (or ER-tree) Hamiltonian
of Eq. (2), the tree tensor network state, its effective Hamiltonians and the
second-order one-site TDVP sweep (the projector-splitting integrator the
paper's Methods section names for its TTNS evolution), plus the observables
the paper plots (electronic populations, reaction-coordinate occupations).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the HIP library and the library never
calls it.

Modules
-------
chain   spectral density -> chain coefficients (closed form, hard cutoff)
model   model description -> tree topology, operators and the term list
ttns    the TTNS state, environments, H_eff, guarded QR, Lanczos expv, sweep
ed      dense Hamiltonians and full state vectors for exact checks on tiny trees

Parity status: every function here is pinned by CPU tests against closed
forms, exact diagonalisation or brute force (see tests/test_oracle_*.py); the
paper itself prints no worked example for this path, so agreement with the
paper's own numbers is "parity unpinned" (its model parameters live in a
supplement that is not available).
"""

"""Energy surfaces of the electronic system (CPU oracle, test infrastructure).

The paper computes its energy surfaces on the fly as the eigenvalues of an
effective Hamiltonian (Eq. 3) and an effective potential (Eq. 4): matrices
of H and of H - T (T the environments' kinetic energy) between the product
states |phi_i>|j> of a bath state phi_i and an electronic state j, where the
bath states come from the singular value decomposition of the wave function
across the system-environment bipartition (at most as many as electronic
states).  With the orthogonality centre at the root, that bipartition is
the root tensor C[sigma, beta] matricised as sigma x (all bonds): C = U S Vh,
and bath state i is row i of Vh in the basis of the isometric subtrees.  The
matrix element is then the root's effective Hamiltonian (the projection of
the operator onto the span of the root's basis) between the root tensors
X_(ij)[sigma, beta] = delta(sigma, j) Vh[i, beta].

Readings: bath states are kept while s_i > rank_tol * s_0 (rank_tol 1e-8),
since the others are not determined by the state; rows and columns are
ordered (i, j) -> i * n_levels + j.
"""
import numpy as np


def bath_states(tt, rank_tol=1e-8):
    """(s, Vh) of the retained bath states, the centre at the root."""
    assert tt.centre == 0
    C = tt.T[0]
    M = C.reshape(C.shape[0], -1)
    _, s, Vh = np.linalg.svd(M, full_matrices=False)
    r = int(np.sum(s > rank_tol * s[0])) if s[0] > 0 else 0
    return s[:r], Vh[:r]


def effective_matrix(tt, rank_tol=1e-8):
    """The (r n) x (r n) matrix <phi_i|<j| H |phi_k>|l> of the TTNS's own
    operator sum (H, or H - T for a tree built with potential=True)."""
    s, Vh = bath_states(tt, rank_tol)
    C = tt.T[0]
    n = C.shape[0]
    r = len(s)
    basis = []
    for i in range(r):
        for j in range(n):
            X = np.zeros((n, Vh.shape[1]), dtype=np.complex128)
            X[j] = Vh[i]
            basis.append(X.reshape(C.shape))
    Hm = np.zeros((r * n, r * n), dtype=np.complex128)
    for b, Xb in enumerate(basis):
        Y = tt.apply_heff(0, Xb)
        for a, Xa in enumerate(basis):
            Hm[a, b] = np.vdot(Xa, Y)
    return Hm, s


def energy_surfaces(tt, rank_tol=1e-8):
    """Eigenvalues (ascending) of effective_matrix."""
    Hm, _ = effective_matrix(tt, rank_tol)
    return np.linalg.eigvalsh(0.5 * (Hm + Hm.conj().T))


def copy_state(dst, src):
    """Put src's state (centre at the root) into dst, a TTNS of the same
    tree and bond dimensions but possibly another operator sum, and build
    dst's environments towards the root."""
    assert src.centre == 0 and [t.shape for t in dst.T] == [t.shape for t in src.T]
    dst.T = [t.copy() for t in src.T]
    dst.centre = 0
    for v in range(dst.n - 1, 0, -1):
        dst.env_update(v, dst.parent[v])

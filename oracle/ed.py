"""Exact references on tiny trees (CPU oracle, test infrastructure).

The Hilbert space is the tensor product of the nodes' physical legs in node
order (ER nodes have dimension 1).  ``dense_hamiltonian`` writes the operator
sum out as a dense matrix; ``embedding`` maps a centre tensor (or a bond
matrix) into the full space through the current isometries, so that
P^H H P is the exact projected Hamiltonian against which H_eff and H_bond are
checked.
"""
import numpy as np

from .ttns import mode_product


def place(ops_at, phys):
    """Kronecker product over all nodes with the given operators placed."""
    out = np.ones((1, 1), dtype=np.complex128)
    for v, d in enumerate(phys):
        op = ops_at.get(v)
        if op is None:
            op = np.eye(d, dtype=np.complex128)
        out = np.kron(out, op)
    return out


def dense_hamiltonian(tree):
    phys = tree.phys
    N = int(np.prod(phys))
    H = np.zeros((N, N), dtype=np.complex128)
    for coef, a, oa, b, ob in tree.terms:
        ops = {a: oa} if b is None else {a: oa, b: ob}
        H += coef * place(ops, phys)
    return H


def initial_full_state(tree):
    psi = np.ones(1, dtype=np.complex128)
    for v in range(len(tree.phys)):
        psi = np.kron(psi, np.asarray(tree.init_local[v], dtype=np.complex128))
    return psi


def embedding_node(ttns, v):
    """Columns: full states obtained by putting unit tensors at node v."""
    saved = ttns.T[v]
    shp = ttns.shape[v]
    cols = []
    for i in range(int(np.prod(shp))):
        e = np.zeros(int(np.prod(shp)), dtype=np.complex128)
        e[i] = 1.0
        ttns.T[v] = e.reshape(shp)
        cols.append(ttns.full_state())
    ttns.T[v] = saved
    return np.array(cols).T


def embedding_bond(ttns, u, v):
    """Full states for unit bond matrices R[a_u, a_v] inserted between an
    isometry u (towards v) and node v's current tensor: the map that defines
    the bond effective Hamiltonian."""
    saved = ttns.T[v]
    ax = ttns.axis_of(v, u)
    Du = ttns.shape[u][ttns.axis_of(u, v)]
    Dv = saved.shape[ax]
    cols = []
    for i in range(Du):
        for j in range(Dv):
            R = np.zeros((Du, Dv), dtype=np.complex128)
            R[i, j] = 1.0
            ttns.T[v] = mode_product(R, saved, ax)
            cols.append(ttns.full_state())
    ttns.T[v] = saved
    return np.array(cols).T

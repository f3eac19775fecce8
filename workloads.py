"""Seeded synthetic workloads for the TTNS one-site TDVP hot path.

This module only draws and lists model parameters (plain numbers and small
matrices).  It performs none of the method's arithmetic: the spectral-density
to chain mapping, the Hamiltonian assembly, the tree construction and the time
evolution all live on the two sides that consume these descriptions (the CPU
oracle and the HIP library), each written independently.

A model description is a dict with these keys:

``h_el``       (n, n) complex   electronic (system) Hamiltonian H_S of Eq. (2)
``init_el``    (n,) complex     initial electronic amplitudes (bath in vacuum)
``chains``     list of dicts    one per bosonic environment i of Eq. (2):
                                ``coupling`` (n, n) complex system operator
                                (the paper's coupling pattern), ``alpha``,
                                ``wc``, ``s`` of the spectral density
                                J(w) = 2 pi alpha wc (w/wc)^s theta(wc - w),
                                chain length ``L``, local dimension ``d``,
                                bond dimension ``D``
               optional ``obb``: size of an optimised boson basis (0: none)
``topology``   "star" (chains hang off the electronic root) or "er" (a binary
               tree of entanglement-renormalisation nodes between the root and
               the chains, Fig. 2 of the paper)
``er_D``       bond dimension on edges between the root and ER nodes
``dt``         time step in the Hamiltonian's inverse energy unit (hbar = 1)
``steps``      number of second-order TDVP steps
``krylov``     Krylov dimension of the local exponentials

Units: the dimensionless spin-boson workloads use hbar = 1 and wc = 1; the
vibronic workloads quote energies in eV and the time step in fs, so ``dt`` is
dt_fs / hbar with hbar in eV fs.
"""
from __future__ import annotations

import numpy as np

HBAR_EV_FS = 0.6582119569509066  # hbar in eV*fs (from the SI-defined h and e)

SIGMA_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIGMA_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def spin_boson(eps=0.0, delta=0.2, alpha=0.1, wc=1.0, s=1.0, L=10, d=10, D=8,
               dt=0.05, steps=200, init=(1.0, 0.0), krylov=12):
    """Spin-boson model as a tree with one chain (basis up, down; sz|up> = +|up>).

    H_S = (eps/2) sz + (delta/2) sx, coupling operator sz.
    """
    h_el = 0.5 * eps * SIGMA_Z + 0.5 * delta * SIGMA_X
    init_el = np.asarray(init, dtype=np.complex128)
    return {
        "name": "spin_boson",
        "h_el": h_el,
        "init_el": init_el,
        "chains": [{"coupling": SIGMA_Z.copy(), "alpha": float(alpha), "wc": float(wc),
                    "s": float(s), "L": int(L), "d": int(d), "D": int(D)}],
        "topology": "star",
        "er_D": int(D),
        "dt": float(dt),
        "steps": int(steps),
        "krylov": int(krylov),
    }


def spin_boson_reference():
    """Single-chain spin-boson workload: eps=0, Delta=0.2, alpha=0.1, wc=1,
    hard cutoff, 10 sites, local dimension 10, bond dimension 8, dt=0.05,
    200 steps, initial state |up> x vacuum."""
    return spin_boson()


def _vibronic_levels(rng, n_levels):
    h = np.zeros((n_levels, n_levels), dtype=np.complex128)
    diag = rng.uniform(0.0, 0.3, size=n_levels)
    for j in range(n_levels):
        h[j, j] = diag[j]
    # off-diagonal couplings: real, N(0, 0.05 eV), upper triangle row-major
    for j in range(n_levels):
        for k in range(j + 1, n_levels):
            v = rng.normal(0.0, 0.05)
            h[j, k] = v
            h[k, j] = v
    return h


def _level_mask(rng, n_levels):
    while True:
        m = rng.integers(0, 2, size=n_levels)
        if m.any():
            return m.astype(np.float64)


def vibronic(seed=2, n_levels=5, n_chains=4, L=40, d=20, D=20, wc=0.2,
             alpha_range=(0.05, 0.2), dt_fs=0.5, steps=400, topology="star",
             er_D=None, krylov=12, init_level=0):
    """Five-state vibronic tree (seeded).

    Diagonal energies U[0, 0.3] eV, off-diagonal couplings N(0, 0.05 eV);
    chain i couples diagonally (0/1 mask, never empty) to a random subset of
    the levels with Ohmic alpha_i in ``alpha_range`` and cutoff ``wc`` (eV).
    The run starts in level ``init_level`` with the bath in vacuum.
    """
    rng = np.random.default_rng(seed)
    h_el = _vibronic_levels(rng, n_levels)
    chains = []
    for _ in range(n_chains):
        alpha = float(rng.uniform(*alpha_range))
        mask = _level_mask(rng, n_levels)
        chains.append({"coupling": np.diag(mask).astype(np.complex128), "alpha": alpha,
                       "wc": float(wc), "s": 1.0, "L": int(L), "d": int(d), "D": int(D)})
    init_el = np.zeros(n_levels, dtype=np.complex128)
    init_el[init_level] = 1.0
    return {
        "name": "vibronic",
        "h_el": h_el,
        "init_el": init_el,
        "chains": chains,
        "topology": topology,
        "er_D": int(er_D if er_D is not None else D),
        "dt": float(dt_fs / HBAR_EV_FS),
        "dt_fs": float(dt_fs),
        "steps": int(steps),
        "krylov": int(krylov),
        "seed": int(seed),
    }


def vibronic_reference():
    """Five-state vibronic tree: 4 chains of 40 sites, d=20, D=20, wc=0.2 eV,
    dt=0.5 fs, 400 steps, seed 2."""
    return vibronic()


def vibronic_small(seed=2, L=6, d=5, D=5, steps=4, n_chains=4):
    """Same recipe as the five-state tree at sizes the oracle finishes fast."""
    return vibronic(seed=seed, L=L, d=d, D=D, steps=steps, n_chains=n_chains)


def large_tree(seed=4, L=100, d=30, D=48, steps=200, krylov=12):
    """Five-state root with 8 chains of 100 sites (d=30, D=48) joined to the
    root through a binary tree of entanglement-renormalisation nodes."""
    return vibronic(seed=seed, n_chains=8, L=L, d=d, D=D, steps=steps,
                    topology="er", er_D=D, krylov=krylov)


def ensemble(seed=3, n=256, steps=100, dt=0.05):
    """Uneven batch of spin-boson instances: L ~ U{20..120}, d in {8,16,24},
    D in {8,16,32}, Delta ~ U[0.1, 1], alpha ~ U[0.01, 0.3]; eps=0, wc=1."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        L = int(rng.integers(20, 121))
        d = int(rng.choice([8, 16, 24]))
        D = int(rng.choice([8, 16, 32]))
        delta = float(rng.uniform(0.1, 1.0))
        alpha = float(rng.uniform(0.01, 0.3))
        out.append(spin_boson(eps=0.0, delta=delta, alpha=alpha, wc=1.0, L=L, d=d, D=D,
                              dt=dt, steps=steps))
    return out


def with_obb(model, obb):
    """The same model with an optimised boson basis of ``obb`` states on
    every chain (chain key ``obb``; 0 removes it)."""
    m = dict(model)
    m["chains"] = [dict(c, obb=int(obb)) for c in model["chains"]]
    return m


def obb_tree(seed=5, L=30, d=40, obb=12, D=12, steps=100):
    """Five-state vibronic tree whose four chains carry an optimised boson
    basis: d Fock states per site behind ``obb`` basis states, chain bond
    dimension D (the paper's run keeps 100 Fock states behind 40 basis
    states and D = 30 along the chains)."""
    return with_obb(vibronic(seed=seed, L=L, d=d, D=D, steps=steps), obb)


def learned_sets(first_seed, count, **kw):
    """Parameter sets of the five-state family used as training / test data
    for the learned propagator (seeds first_seed .. first_seed+count-1)."""
    return [vibronic(seed=first_seed + k, **kw) for k in range(count)]


def chain_count(model):
    return len(model["chains"])


def node_count(model):
    """Number of tree nodes (root + ER nodes + chain sites, and one basis
    node per site of a chain with an optimised boson basis)."""
    n = 1 + sum(c["L"] * (2 if c.get("obb", 0) else 1) for c in model["chains"])
    if model["topology"] == "er":
        n += er_node_count(len(model["chains"]))
    return n


def er_node_count(n_chains):
    """ER nodes of the balanced binary tree that joins the chain heads (its
    leaves, in chain order) to the electronic root: the root carries the two
    halves of the chain list, and every group of more than one chain hangs
    below one ER node whose two children carry the halves of that group."""
    def group(n):
        return 0 if n <= 1 else 1 + group((n + 1) // 2) + group(n // 2)
    if n_chains <= 1:
        return 0
    return group((n_chains + 1) // 2) + group(n_chains // 2)

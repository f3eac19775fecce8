"""Model description -> tree, operators and Hamiltonian terms (CPU oracle).

Builds the star Hamiltonian of Eq. (2),

    H = H_S + sum_i [ A_i (x) c0_i (a_i0^+ + a_i0) + H_chain,i ],

as an operator sum over tree nodes ("tree MPO").  The coupling operator A_i
plays the role of the paper's pattern W_i with its strength absorbed into the
chain coefficient c0_i (our reading: c0 comes from the spectral density).

Tree layout (nodes numbered in pre-order, children in order):
* node 0 is the electronic root (physical dimension = number of levels);
* topology "star": chain i hangs directly below the root, site n's only
  child is site n+1;
* with an optimised boson basis (chain key ``obb`` > 0, Methods "Tensor
  Network States"), site n has no physical leg and two children: a basis
  node holding the d Fock states of the site behind a bond of dimension
  ``obb`` (the d -> obb basis tensor), then site n+1; the boson operators of
  the site act on its basis node;
* topology "er": the chain heads are joined to the root through a balanced
  binary tree of entanglement-renormalisation nodes (physical dimension 1),
  the construction Fig. 2 of the paper uses to avoid the order-(N+1) root.

Each term is (coef, node_a, op_a, node_b, op_b) with node_b = None for an
on-site term; hermitian conjugate pairs are listed explicitly.
"""
import numpy as np

from .chain import ohmic_chain


def boson_ops(d):
    """Truncated boson operators on |0..d-1>: b|k> = sqrt(k)|k-1>."""
    b = np.zeros((d, d), dtype=np.complex128)
    for k in range(1, d):
        b[k - 1, k] = np.sqrt(k)
    bd = b.conj().T.copy()
    num = np.diag(np.arange(d, dtype=np.float64)).astype(np.complex128)
    return b, bd, num


class TreeModel:
    """Topology, dims, requested bond dims, terms and initial local states."""

    def __init__(self):
        self.parent = []
        self.phys = []
        self.bond_req = []
        self.init_local = []
        self.terms = []          # (coef, a, op_a, b, op_b)
        self.heads = []          # node index of every chain head, chain order
        self.chain_nodes = []    # list of node lists per chain
        self.kind = []           # "el", "er", "site"

    def add_node(self, parent, d, D, local, kind):
        self.parent.append(parent)
        self.phys.append(int(d))
        self.bond_req.append(int(D))
        self.init_local.append(np.asarray(local, dtype=np.complex128))
        self.kind.append(kind)
        return len(self.parent) - 1


def momentum_op(d):
    """p = i (b^+ - b) / sqrt(2) on |0..d-1> (Hermitian)."""
    b, bd, _ = boson_ops(d)
    return 1j * (bd - b) / np.sqrt(2.0)


def build_tree(model, potential=False):
    """Translate a workload description into a TreeModel.

    With ``potential`` the operator sum is H - T instead of H, T the kinetic
    energy of the environments' normal modes: for a chain with site energies
    eps_n and hoppings t_n (the tridiagonal matrix M of its modes),
    sum_modes (w/2) P^2 = (1/2) p^T M p with p_n = i (b_n^+ - b_n)/sqrt(2)
    the chain-site momenta, i.e. the on-site terms (eps_n/2) p_n^2 and the
    pair terms t_n p_n p_{n+1}.  Eq. (4)'s effective potential is built from
    this operator (also selected by a true ``potential`` key of the model)."""
    potential = potential or bool(model.get("potential", False))
    tm = TreeModel()
    h_el = np.asarray(model["h_el"], dtype=np.complex128)
    n_el = h_el.shape[0]
    tm.add_node(-1, n_el, 0, model["init_el"], "el")
    tm.terms.append((1.0, 0, h_el, None, None))
    chains = model["chains"]
    tm.heads = [None] * len(chains)
    tm.chain_nodes = [None] * len(chains)

    def add_chain(i, p):
        ch = chains[i]
        d, D, L = ch["d"], ch["D"], ch["L"]
        obb = int(ch.get("obb", 0))
        c0, eps, t = ohmic_chain(ch["alpha"], ch["wc"], ch.get("s", 1.0), L)
        b, bd, num = boson_ops(d)
        vac = np.zeros(d, dtype=np.complex128)
        vac[0] = 1.0
        nodes = []
        prev = p
        for n in range(L):
            if obb:
                # optimised boson basis: the site carries no physical leg; its
                # first child holds the d Fock states behind a bond of
                # dimension obb (the basis tensor), its second the next site
                site = tm.add_node(prev, 1, D, [1.0], "site")
                node = tm.add_node(site, d, obb, vac, "obb")
                prev = site
            else:
                node = tm.add_node(prev, d, D, vac, "site")
                prev = node
            nodes.append(node)
        tm.heads[i] = nodes[0]
        tm.chain_nodes[i] = nodes
        A = np.asarray(ch["coupling"], dtype=np.complex128)
        tm.terms.append((c0, 0, A, nodes[0], b + bd))
        for n in range(L):
            tm.terms.append((eps[n], nodes[n], num, None, None))
        for n in range(L - 1):
            tm.terms.append((t[n], nodes[n], bd, nodes[n + 1], b))
            tm.terms.append((t[n], nodes[n], b, nodes[n + 1], bd))
        if potential:
            p = momentum_op(d)
            for n in range(L):
                tm.terms.append((-0.5 * eps[n], nodes[n], p @ p, None, None))
            for n in range(L - 1):
                tm.terms.append((-t[n], nodes[n], p, nodes[n + 1], p))

    def group(p, idx):
        if len(idx) == 1:
            add_chain(idx[0], p)
            return
        e = tm.add_node(p, 1, model["er_D"], [1.0], "er")
        half = (len(idx) + 1) // 2
        group(e, idx[:half])
        group(e, idx[half:])

    order = list(range(len(chains)))
    if model["topology"] == "star" or len(chains) <= 1:
        for i in order:
            add_chain(i, 0)
    elif model["topology"] == "er":
        half = (len(order) + 1) // 2
        group(0, order[:half])
        group(0, order[half:])
    else:
        raise ValueError("unknown topology %r" % model["topology"])
    return tm

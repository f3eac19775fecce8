"""Tree tensor network state and its one-site TDVP integrator (CPU oracle).

Plain complex128 NumPy, written for checkability rather than speed.

State.  One tensor per node.  Axis order of node v: [parent bond] (absent at
the root), physical leg, child bonds in child order.  Away from the centre,
every node is an isometry towards the centre.

Time evolution.  The paper evolves its TTNS with the time-dependent
variational principle: each tensor in turn is evolved with a local effective
Hamiltonian built from the full state (section "TTNS for vibronic quantum
dynamics"; Methods).  We use the one-site projector-splitting integrator of
Lubich-Oseledets (2014) / Haegeman et al. (2016) that the paper cites, in its
tree form: every node is evolved forward with exp(-i h H_eff) and every bond
matrix backward with exp(+i h H_bond), visiting the tree depth first.  One
second-order step of size dt = pre-order sweep with h = dt/2 followed by its
adjoint, a post-order sweep with h = dt/2.

Readings where the paper is silent (its TDVP details are in an unavailable
supplement):
* bond dimensions larger than either side's Hilbert space are clamped;
* rank-deficient QR factors are completed deterministically (``qr_guarded``);
* local exponentials use Lanczos with classical Gram-Schmidt applied twice,
  Krylov dimension m (12), breakdown when beta_j <= 1e-12 |x|;
* the turnaround leaf is evolved twice with h (no merging).
"""
import numpy as np
from scipy.linalg import eigh_tridiagonal

PHYS = "phys"


# ----------------------------------------------------------------------------
# small tensor helpers
# ----------------------------------------------------------------------------

def mode_product(M, X, axis):
    """Y[.., a', ..] = sum_a M[a', a] X[.., a, ..] on the given axis."""
    return np.moveaxis(np.tensordot(M, X, axes=([1], [axis])), 0, axis)


def matricize(X, axis):
    """Rows: all other axes (row-major, original order); columns: ``axis``."""
    return np.moveaxis(X, axis, -1).reshape(-1, X.shape[axis])


def unmatricize(Mat, shape, axis):
    rest = [shape[i] for i in range(len(shape)) if i != axis]
    return np.moveaxis(Mat.reshape(rest + [shape[axis]]), -1, axis)


def completion_order(shape, axis, phys_axis):
    """Row indices of matricize(X, axis) enumerated with the physical index
    fastest, then the remaining bond axes in axis order (each next slower)."""
    rem = [i for i in range(len(shape)) if i != axis]
    others = [i for i in rem if i != phys_axis]
    counter_axes = [phys_axis] + others          # fastest first
    dims_fast_first = [shape[i] for i in counter_axes]
    total = int(np.prod(dims_fast_first)) if dims_fast_first else 1
    n = np.arange(total)
    idx = {}
    for ax, dim in zip(counter_axes, dims_fast_first):
        idx[ax] = n % dim
        n = n // dim
    rem_dims = [shape[i] for i in rem]
    return np.ravel_multi_index(tuple(idx[i] for i in rem), rem_dims)


def qr_guarded(A, order, rank_tol):
    """QR of A (rows x cols) column by column, with a deterministic completion.

    Column k: project out the previous Q columns twice (classical Gram-Schmidt
    applied twice).  If the residual norm exceeds rank_tol * |A|_F the column
    is normalised (so R_kk is real and positive: the QR is unique for full
    rank).  Otherwise Q_k is the first unit vector e_i, i taken in ``order``,
    whose squared distance from span(Q_0..Q_{k-1}) exceeds half its average
    over all unit vectors, (rows - k) / (2 rows) -- the largest distance
    always does -- orthogonalised twice against the previous columns; R_kk is
    then the projection of the residual on Q_k.  A = Q R up to the dropped
    residuals.  Returns (Q, R, number of completed columns).
    """
    rows, cols = A.shape
    Q = np.zeros((rows, cols), dtype=np.complex128)
    R = np.zeros((cols, cols), dtype=np.complex128)
    tol = rank_tol * np.linalg.norm(A)
    guarded = 0
    for k in range(cols):
        Qk = Q[:, :k]
        a = A[:, k]
        h1 = Qk.conj().T @ a
        v = a - Qk @ h1
        h2 = Qk.conj().T @ v
        v = v - Qk @ h2
        R[:k, k] = h1 + h2
        r = np.linalg.norm(v)
        if r > tol:
            Q[:, k] = v / r
            R[k, k] = r
            continue
        guarded += 1
        chosen = None
        comp_tol = 0.5 * (rows - k) / rows
        for i in order:
            if 1.0 - np.sum(np.abs(Qk[i, :]) ** 2) > comp_tol:
                chosen = i
                break
        if chosen is None:
            raise RuntimeError("qr_guarded: no completion vector available")
        u = np.zeros(rows, dtype=np.complex128)
        u[chosen] = 1.0
        u = u - Qk @ (Qk.conj().T @ u)
        u = u - Qk @ (Qk.conj().T @ u)
        u = u / np.linalg.norm(u)
        Q[:, k] = u
        R[k, k] = np.vdot(u, v)
    return Q, R, guarded


def expv(apply, x, z, m, breakdown_tol=1e-12, info=None):
    """exp(z H) x by Lanczos (H Hermitian, given as ``apply``).

    v_1 = x/|x|; w = H v_j orthogonalised against all v_i by classical
    Gram-Schmidt applied twice; alpha_j = Re<v_j|H v_j>, beta_j = |w|.
    Stops at j = m, at j = dim(x) or when beta_j <= breakdown_tol |x|.
    Result |x| V exp(z T) e_1 with T the real symmetric tridiagonal matrix,
    exponentiated through its eigendecomposition.
    """
    nx = np.linalg.norm(x)
    if nx == 0.0:
        return x.copy()
    N = x.size
    V = [x / nx]
    alpha, beta = [], []
    kmax = min(m, N)
    for j in range(kmax):
        w = apply(V[j])
        Vm = np.array(V)
        h1 = Vm.conj() @ w
        w = w - h1 @ Vm
        h2 = Vm.conj() @ w
        w = w - h2 @ Vm
        alpha.append((h1[j] + h2[j]).real)
        if j == kmax - 1:
            if info is not None:
                info["last_beta"] = np.linalg.norm(w)
            break
        b = np.linalg.norm(w)
        if b <= breakdown_tol * nx:
            if info is not None:
                info["breakdown"] = info.get("breakdown", 0) + 1
            break
        beta.append(b)
        V.append(w / b)
    k = len(alpha)
    if k == 1:
        coef = np.array([np.exp(z * alpha[0])])
    else:
        evals, evecs = eigh_tridiagonal(np.array(alpha), np.array(beta))
        coef = evecs @ (np.exp(z * evals) * evecs[0, :])
    return nx * (coef @ np.array(V[:k]))


# ----------------------------------------------------------------------------
# the TTNS
# ----------------------------------------------------------------------------

def clamp_bond_dims(parent, phys, bond_req, children):
    """Clamp every bond to the Hilbert-space dimension reachable on each side
    through the neighbouring node (iterated to a fixed point)."""
    n = len(parent)
    D = [0] + [max(1, int(bond_req[v])) for v in range(1, n)]
    changed = True
    while changed:
        changed = False
        for v in range(n - 1, 0, -1):
            cap = phys[v]
            for c in children[v]:
                cap *= D[c]
            if D[v] > cap:
                D[v] = cap
                changed = True
        for v in range(1, n):
            p = parent[v]
            cap = phys[p] * (D[p] if p != 0 else 1)
            for s in children[p]:
                if s != v:
                    cap *= D[s]
            if D[v] > cap:
                D[v] = cap
                changed = True
    return D


class TTNS:
    def __init__(self, tree, krylov=12, rank_tol=1e-8, breakdown_tol=1e-12):
        self.tree = tree
        self.parent = list(tree.parent)
        self.phys = list(tree.phys)
        self.n = len(self.parent)
        self.terms = list(tree.terms)
        self.krylov = krylov
        self.rank_tol = rank_tol
        self.breakdown_tol = breakdown_tol
        self.stats = {"guarded": 0, "breakdown": 0, "node_updates": 0}
        n = self.n
        self.children = [[] for _ in range(n)]
        for v in range(1, n):
            assert 0 <= self.parent[v] < v, "parents must precede children"
            self.children[self.parent[v]].append(v)
        # pre-order numbering => subtree(v) = [v, v + size[v])
        self.size = [1] * n
        for v in range(n - 1, 0, -1):
            self.size[self.parent[v]] += self.size[v]
        for v in range(n):
            for c in self.children[v]:
                assert c < v + self.size[v]
        self.D = clamp_bond_dims(self.parent, self.phys, tree.bond_req, self.children)
        # axes
        self.nbrs = [([self.parent[v]] if v else []) + self.children[v] for v in range(n)]
        self.phys_axis = [0 if v == 0 else 1 for v in range(n)]
        self.shape = []
        for v in range(n):
            dims = ([self.D[v]] if v else []) + [self.phys[v]] + [self.D[c] for c in self.children[v]]
            self.shape.append(tuple(dims))
        self.env = {}
        self._plans = {}
        self._chan = {}
        self._bond_terms = {}
        self._init_state(tree.init_local)
        self.centre = 0
        for v in range(n - 1, 0, -1):
            self.env_update(v, self.parent[v])

    # -- topology ------------------------------------------------------------
    def axis_of(self, v, u):
        if u == PHYS:
            return self.phys_axis[v]
        if v != 0 and u == self.parent[v]:
            return 0
        return self.phys_axis[v] + 1 + self.children[v].index(u)

    def in_subtree(self, n, v):
        return v <= n < v + self.size[v]

    def region(self, v, node):
        """Where ``node`` sits as seen from v: PHYS, or the neighbour of v on
        the path towards it."""
        if node == v:
            return PHYS
        if self.in_subtree(node, v):
            for c in self.children[v]:
                if self.in_subtree(node, c):
                    return c
        return self.parent[v]

    def in_side(self, node, u, v):
        """Is ``node`` on u's side of the edge (u, v)?"""
        if v == self.parent[u]:
            return self.in_subtree(node, u)
        return not self.in_subtree(node, v)

    def path(self, a, b):
        """Node sequence from a to b."""
        up_a, up_b = [a], [b]
        while up_a[-1] != 0:
            up_a.append(self.parent[up_a[-1]])
        while up_b[-1] != 0:
            up_b.append(self.parent[up_b[-1]])
        sa = set(up_a)
        lca = next(x for x in up_b if x in sa)
        p1 = up_a[:up_a.index(lca) + 1]
        p2 = up_b[:up_b.index(lca)]
        return p1 + p2[::-1]

    def last_preorder_leaf(self, v):
        return v + self.size[v] - 1

    # -- initial state -------------------------------------------------------
    def _init_state(self, init_local):
        self.T = [None] * self.n
        for v in range(self.n):
            loc = np.asarray(init_local[v], dtype=np.complex128)
            shp = self.shape[v]
            if v == 0:
                C = np.zeros(shp, dtype=np.complex128)
                idx = (slice(None),) + (0,) * (len(shp) - 1)
                C[idx] = loc
                self.T[0] = C
                continue
            # isometry towards the parent: column 0 = local (x) child states 0,
            # remaining columns completed in the physical-fastest order
            col = np.zeros(shp[1:], dtype=np.complex128)
            col[(slice(None),) + (0,) * (len(shp) - 2)] = loc
            A = np.zeros((int(np.prod(shp[1:])), shp[0]), dtype=np.complex128)
            A[:, 0] = col.reshape(-1)
            order = completion_order(shp, 0, 1)
            Q, _, _ = qr_guarded(A, order, self.rank_tol)
            self.T[v] = unmatricize(Q, shp, 0)

    # -- environments ----------------------------------------------------------
    def channels(self, u, v):
        """Channel keys of the environment of u's side seen from v: the block
        Hamiltonian "H" and one (term, end) key per two-node term with exactly
        one end on u's side."""
        if (u, v) in self._chan:
            return self._chan[(u, v)]
        keys = ["H"]
        for k, (coef, a, oa, b, ob) in enumerate(self.terms):
            if b is None:
                continue
            ia, ib = self.in_side(a, u, v), self.in_side(b, u, v)
            if ia and not ib:
                keys.append((k, 0))
            elif ib and not ia:
                keys.append((k, 1))
        self._chan[(u, v)] = keys
        return keys

    def _factor(self, v, region, k, end, op, X):
        if region == PHYS:
            return mode_product(op, X, self.phys_axis[v])
        return mode_product(self.env[(region, v)][(k, end)], X, self.axis_of(v, region))

    def _plan(self, v, exclude):
        """Terms of the operator summed by ``_local_sum`` (cached per node)."""
        key = (v, exclude)
        if key not in self._plans:
            site, pairs = [], []
            for k, (coef, a, oa, b, ob) in enumerate(self.terms):
                if b is None:
                    if a == v:
                        site.append((coef, oa))
                    continue
                ra, rb = self.region(v, a), self.region(v, b)
                if ra == rb or ra == exclude or rb == exclude:
                    continue
                pairs.append((coef, k, ra, oa, rb, ob))
            envs = [w for w in self.nbrs[v] if w != exclude]
            self._plans[key] = (site, pairs, envs)
        return self._plans[key]

    def _local_sum(self, v, X, exclude):
        """Apply (sum of H terms acting inside v's region set) to X, where the
        regions of v are its physical leg and its neighbour sides except
        ``exclude`` (None: all neighbours = H_eff at v).  Terms with both ends
        inside one neighbour side are already in that side's H channel."""
        site, pairs, envs = self._plan(v, exclude)
        Y = np.zeros_like(X)
        for coef, op in site:
            Y += coef * mode_product(op, X, self.phys_axis[v])
        for coef, k, ra, oa, rb, ob in pairs:
            Y += coef * self._factor(v, ra, k, 0, oa, self._factor(v, rb, k, 1, ob, X))
        for w in envs:
            Y += mode_product(self.env[(w, v)]["H"], X, self.axis_of(v, w))
        return Y

    def env_update(self, u, v):
        """E_{u->v}: every channel of u's side, in the basis of u's isometry."""
        T = self.T[u]
        ax = self.axis_of(u, v)
        Tm = matricize(T, ax).conj().T
        out = {}
        for key in self.channels(u, v):
            if key == "H":
                X = self._local_sum(u, T, exclude=v)
            else:
                k, end = key
                term = self.terms[k]
                node = term[1] if end == 0 else term[3]
                op = term[2] if end == 0 else term[4]
                X = self._factor(u, self.region(u, node), k, end, op, T)
            out[key] = Tm @ matricize(X, ax)
        self.env[(u, v)] = out

    # -- effective Hamiltonians ------------------------------------------------
    def apply_heff(self, v, C):
        return self._local_sum(v, C, exclude=None)

    def apply_hbond(self, u, v, R):
        """H_bond R for the bond matrix R[a_u, a_v] between u and v."""
        Eu, Ev = self.env[(u, v)], self.env[(v, u)]
        if (u, v) not in self._bond_terms:
            cross = []
            for k, (coef, a, oa, b, ob) in enumerate(self.terms):
                if b is None:
                    continue
                ia = self.in_side(a, u, v)
                ib = self.in_side(b, u, v)
                if ia == ib:
                    continue
                cross.append((coef, k) + ((0, 1) if ia else (1, 0)))
            self._bond_terms[(u, v)] = cross
        Y = Eu["H"] @ R + R @ Ev["H"].T
        for coef, k, eu, ev in self._bond_terms[(u, v)]:
            Y = Y + coef * (Eu[(k, eu)] @ R @ Ev[(k, ev)].T)
        return Y

    # -- elementary sweep operations ------------------------------------------
    def evolve_node(self, v, h):
        shp = self.shape[v]
        info = {}
        f = lambda x: self.apply_heff(v, x.reshape(shp)).reshape(-1)
        self.T[v] = expv(f, self.T[v].reshape(-1), -1j * h, self.krylov,
                         self.breakdown_tol, info).reshape(shp)
        self.stats["breakdown"] += info.get("breakdown", 0)
        self.stats["node_updates"] += 1

    def qr_to(self, u, v):
        """Make u an isometry towards its neighbour v; return the bond matrix."""
        ax = self.axis_of(u, v)
        shp = self.shape[u]
        Q, R, g = qr_guarded(matricize(self.T[u], ax),
                             completion_order(shp, ax, self.phys_axis[u]), self.rank_tol)
        self.stats["guarded"] += g
        self.T[u] = unmatricize(Q, shp, ax)
        self.env_update(u, v)
        return R

    def absorb(self, u, v, R):
        self.T[v] = mode_product(R, self.T[v], self.axis_of(v, u))
        self.centre = v

    def move(self, u, v, h=None):
        """Centre u -> neighbour v; with h, evolve the bond backward by h."""
        assert self.centre == u
        R = self.qr_to(u, v)
        if h is not None:
            shp = R.shape
            f = lambda x: self.apply_hbond(u, v, x.reshape(shp)).reshape(-1)
            info = {}
            R = expv(f, R.reshape(-1), 1j * h, self.krylov, self.breakdown_tol,
                     info).reshape(shp)
            self.stats["breakdown"] += info.get("breakdown", 0)
        self.absorb(u, v, R)

    def move_to(self, target):
        p = self.path(self.centre, target)
        for a, b in zip(p[:-1], p[1:]):
            self.move(a, b)

    # -- the sweep ---------------------------------------------------------------
    def pre(self, v, h):
        self.evolve_node(v, h)
        ch = self.children[v]
        for i, c in enumerate(ch):
            self.move(v, c, h)
            self.pre(c, h)
            if i < len(ch) - 1:
                self.move_to(v)

    def post(self, v, h):
        ch = self.children[v]
        for i in range(len(ch) - 1, -1, -1):
            c = ch[i]
            if i < len(ch) - 1:
                self.move_to(self.last_preorder_leaf(c))
            self.post(c, h)
            self.move(c, v, h)
        self.evolve_node(v, h)

    def step(self, dt):
        """One second-order TDVP step (centre at the root on entry and exit)."""
        assert self.centre == 0
        self.pre(0, 0.5 * dt)
        self.post(0, 0.5 * dt)

    # -- observables (centre at the root) ---------------------------------------
    def rdm(self):
        """Reduced density matrix of the root's physical leg."""
        C = self.T[0]
        M = C.reshape(C.shape[0], -1)
        return M @ M.conj().T

    def norm2(self):
        return float(np.vdot(self.T[0], self.T[0]).real)

    def energy(self):
        C = self.T[0]
        return float(np.vdot(C, self.apply_heff(0, C)).real)

    def local_expectation(self, node, op):
        """<psi| op_node |psi> with the centre at the root."""
        assert self.centre == 0
        T = self.T[node]
        ax = 0
        M = matricize(T, ax).conj().T @ matricize(mode_product(op, T, self.phys_axis[node]), ax)
        v = node
        while self.parent[v] != 0:
            p = self.parent[v]
            Tp = self.T[p]
            M = matricize(Tp, 0).conj().T @ matricize(mode_product(M, Tp, self.axis_of(p, v)), 0)
            v = p
        C = self.T[0]
        return complex(np.vdot(C, mode_product(M, C, self.axis_of(0, v))))

    def bond_entropy(self, v):
        """Von Neumann entropy of the bipartition (subtree of v | rest):
        with the centre moved to v, the Schmidt values across v's parent bond
        are the singular values of C_v matricised towards the parent axis
        (everything outside is an isometry in the parent index, everything
        below in v's other legs).  Leaves the centre at v."""
        assert v != 0
        self.move_to(v)
        s = np.linalg.svd(matricize(self.T[v], self.axis_of(v, self.parent[v])), compute_uv=False)
        p = s ** 2 / np.sum(s ** 2)
        p = p[p > 1e-300]
        return float(-np.sum(p * np.log(p)))

    def full_state(self):
        """Contract the tree into the full state vector (tiny trees only);
        the index order is the node order, physical legs only."""
        def sub(v):
            X = self.T[v]
            pos = self.phys_axis[v] + 1
            for c in self.children[v]:
                X = np.tensordot(X, sub(c), axes=([pos], [0]))
            if v == 0:
                return X.reshape(-1)
            return X.reshape(X.shape[0], -1)
        return sub(0)


def run(model, steps=None, dt=None, record=True, ttns=None):
    """Evolve a workload; returns (ttns, history) where history holds the
    root reduced density matrices, norms, energies and head occupations at
    t_k = k dt, k = 0..steps."""
    from .model import build_tree, boson_ops
    if ttns is None:
        tree = build_tree(model)
        ttns = TTNS(tree, krylov=model.get("krylov", 12))
    steps = model["steps"] if steps is None else steps
    dt = model["dt"] if dt is None else dt
    heads = ttns.tree.heads
    nums = [boson_ops(model["chains"][i]["d"])[2] for i in range(len(heads))]

    hist = {"rdm": [], "norm": [], "energy": [], "occ": []}

    def rec():
        hist["rdm"].append(ttns.rdm())
        hist["norm"].append(ttns.norm2())
        hist["energy"].append(ttns.energy())
        hist["occ"].append([ttns.local_expectation(h, nums[i]).real for i, h in enumerate(heads)])

    if record:
        rec()
    for _ in range(steps):
        ttns.step(dt)
        if record:
            rec()
    for k in hist:
        hist[k] = np.array(hist[k])
    return ttns, hist

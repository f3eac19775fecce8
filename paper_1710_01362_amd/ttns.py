"""Thin ctypes binding of libttns.so (include/ttns.h).

Argument marshalling only: every step of the TDVP path runs in the HIP
library.  PyTorch provides the device workspace (one uint8 tensor) and the
stream.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttns.so")

TTNS_OK = 0
TTNS_EINVAL = -1
TTNS_ENOMEM = -2
TTNS_EDEVICE = -3
TTNS_ENUMERIC = -4

TTNS_FP64, TTNS_FP32, TTNS_BF16X3 = 0, 1, 2
TTNS_EXEC_AUTO, TTNS_EXEC_WIDE, TTNS_EXEC_PERSISTENT = 0, 1, 2
TTNS_FLAG_MFMA_ALL = 1
TTNS_FLAG_AUTOTUNE = 2

OBS_RDM, OBS_POP, OBS_LOCAL, OBS_NORM, OBS_ENERGY = 0, 1, 2, 3, 4
OBS_HISTORY, OBS_RECORD_SIZE, OBS_TENSOR, OBS_STATS, OBS_BOND_DIMS = 5, 6, 7, 8, 9
OBS_STEP_FLOPS = 10
OBS_ENTROPY = 11

EXPORTED = [
    "ttns_default_opts", "ttns_ohmic_chain", "ttns_workspace_size", "ttns_star_workspace_size",
    "ttns_build", "ttns_star_build", "ttns_apply_heff", "ttns_tdvp_step", "ttns_observe",
    "ttns_profile", "ttns_profile_read", "ttns_profile_kernel", "ttns_tuning_report", "ttns_destroy",
    "ttns_last_error", "ttns_star_build_noalloc", "ttns_struct_sizes", "ttns_energy_surfaces",
    "ttns_copy_state",
]
# kernel ids (include/ttns.h) -> device symbol
KERNELS = {0: "ttns::k_op<0> (scalar apply)", 1: "ttns::k_op<1> (scalar H_eff + Lanczos dots)",
           2: "ttns::k_op<2> (norm)", 3: "ttns::k_op<3> (scale)", 4: "ttns::k_op<4> (Gram-Schmidt 1)",
           5: "ttns::k_op<5> (Gram-Schmidt 2)", 6: "ttns::k_op<6> (Krylov exp + combine)",
           7: "ttns::k_op<7> (guarded QR)", 8: "ttns::k_op<8> (environment contraction)",
           9: "ttns::k_op<9> (bond exponential)", 10: "ttns::k_op<10> (copy)", 11: "ttns::k_op<11> (dot)",
           12: "ttns::k_op<12> (record)", 14: "ttns::k_op<14> (wide QR phase)",
           16: "ttns::k_mode<0> (FP64 MFMA H_eff group)", 17: "ttns::k_mode<1> (FP32 MFMA H_eff group)",
           18: "ttns::k_mode<2> (BF16x3 MFMA H_eff group)"}


class c64(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Term(C.Structure):
    _fields_ = [("node_a", C.c_int32), ("op_a", C.c_int32), ("node_b", C.c_int32),
                ("op_b", C.c_int32), ("coef", C.c_double)]


class Tree(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("parent", C.POINTER(C.c_int32)),
                ("phys_dim", C.POINTER(C.c_int32)), ("bond_dim", C.POINTER(C.c_int32)),
                ("n_ops", C.c_int32), ("op_dim", C.POINTER(C.c_int32)),
                ("op_data", C.POINTER(c64)), ("n_terms", C.c_int32),
                ("terms", C.POINTER(Term)), ("init_local", C.POINTER(c64)),
                ("n_observe", C.c_int32), ("observe_node", C.POINTER(C.c_int32)),
                ("observe_op", C.POINTER(C.c_int32))]


class StarModel(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("h_el", C.POINTER(c64)), ("init_el", C.POINTER(c64)),
                ("n_chains", C.c_int32), ("coupling", C.POINTER(c64)),
                ("alpha", C.POINTER(C.c_double)), ("wc", C.POINTER(C.c_double)),
                ("s", C.POINTER(C.c_double)), ("length", C.POINTER(C.c_int32)),
                ("local_dim", C.POINTER(C.c_int32)), ("bond_dim", C.POINTER(C.c_int32)),
                ("topology", C.c_int32), ("er_bond_dim", C.c_int32),
                ("obb_dim", C.POINTER(C.c_int32)), ("potential", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("krylov_dim", C.c_int32),
                ("breakdown_tol", C.c_double), ("rank_tol", C.c_double),
                ("record_capacity", C.c_int32), ("executor", C.c_int32), ("flags", C.c_uint32)]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # share PyTorch's HIP runtime: map it before libttns.so resolves its
        # libamdhip64 dependency, so workspace, streams and kernels live in one
        # runtime instance
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libttns.so is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P, I, D, S = C.c_void_p, C.c_int32, C.c_double, C.c_size_t
        L.ttns_default_opts.argtypes = [C.POINTER(Opts)]
        L.ttns_default_opts.restype = None
        L.ttns_ohmic_chain.argtypes = [D, D, D, I, C.POINTER(D), C.POINTER(D), C.POINTER(D)]
        L.ttns_workspace_size.argtypes = [C.POINTER(Tree), I, C.POINTER(Opts), C.POINTER(S)]
        L.ttns_star_workspace_size.argtypes = [C.POINTER(StarModel), I, C.POINTER(Opts), C.POINTER(S)]
        L.ttns_build.argtypes = [C.POINTER(Tree), I, C.POINTER(Opts), P, S, P, C.POINTER(P)]
        L.ttns_star_build.argtypes = [C.POINTER(StarModel), I, C.POINTER(Opts), P, S, P, C.POINTER(P)]
        L.ttns_star_build_noalloc.argtypes = [C.POINTER(StarModel), I, C.POINTER(Opts), P, C.POINTER(P)]
        L.ttns_apply_heff.argtypes = [P, I, I, P, P]
        L.ttns_tdvp_step.argtypes = [P, D, I]
        L.ttns_observe.argtypes = [P, I, I, I, C.POINTER(D), S]
        L.ttns_profile.argtypes = [P, I]
        L.ttns_profile_read.argtypes = [P, I, C.POINTER(D), C.POINTER(C.c_int64), C.POINTER(D)]
        L.ttns_profile_kernel.argtypes = [P, I, C.POINTER(D), C.POINTER(C.c_int64), C.POINTER(D), C.POINTER(D)]
        L.ttns_tuning_report.argtypes = [P, C.c_char_p, S, C.POINTER(S)]
        L.ttns_destroy.argtypes = [P]
        L.ttns_last_error.argtypes = [P]
        L.ttns_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("ttns_default_opts", "ttns_last_error"):
                getattr(L, name).restype = C.c_int
        L.ttns_struct_sizes.argtypes = [C.POINTER(S), I]
        L.ttns_energy_surfaces.argtypes = [P, I, D, C.POINTER(I), C.POINTER(D), C.POINTER(D), S]
        L.ttns_copy_state.argtypes = [P, I, P, I]
        _check_struct_sizes(L)
        _lib = L
    return _lib


def _check_struct_sizes(L):
    """Refuse a library compiled from other headers than this binding's
    struct layouts (a stale libttns.so would read the arguments wrongly)."""
    from . import ttnn
    mine = [C.sizeof(c64), C.sizeof(Term), C.sizeof(Tree), C.sizeof(StarModel), C.sizeof(Opts),
            C.sizeof(ttnn.Config)]
    theirs = (C.c_size_t * len(mine))()
    if L.ttns_struct_sizes(theirs, len(mine)) != TTNS_OK or list(theirs) != mine:
        raise RuntimeError("libttns.so was built from other headers than this binding (struct sizes %s vs %s): "
                           "rebuild it" % (list(theirs), mine))


class TTNSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("ttns error %d: %s" % (code, msg))
        self.code = code


def check(rc):
    if rc != TTNS_OK:
        raise TTNSError(rc, lib().ttns_last_error(None).decode())


def default_opts(**kw):
    o = Opts()
    lib().ttns_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def ttns_ohmic_chain(alpha, wc, s, L):
    c0 = C.c_double()
    eps = (C.c_double * L)()
    hop = (C.c_double * max(L - 1, 1))()
    check(lib().ttns_ohmic_chain(alpha, wc, s, L, C.byref(c0), eps, hop))
    return c0.value, np.array(eps[:]), np.array(hop[:L - 1])


def _c64_array(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128).reshape(-1))
    arr = (c64 * max(a.size, 1))()
    view = np.frombuffer(arr, dtype=np.complex128, count=a.size)
    view[:] = a
    return arr


def _arr(ctype, values):
    values = list(values)
    return (ctype * max(len(values), 1))(*values)


def star_model(m, keep):
    """Marshal a workload description (see workloads.py) into a StarModel;
    ``keep`` collects the ctypes buffers that must outlive the call."""
    n = m["h_el"].shape[0]
    ch = m["chains"]
    bufs = {
        "h": _c64_array(m["h_el"]),
        "i": _c64_array(m["init_el"]),
        "A": _c64_array(np.concatenate([np.asarray(c["coupling"]).reshape(-1) for c in ch]) if ch else [0]),
        "al": _arr(C.c_double, [c["alpha"] for c in ch]),
        "wc": _arr(C.c_double, [c["wc"] for c in ch]),
        "s": _arr(C.c_double, [c.get("s", 1.0) for c in ch]),
        "L": _arr(C.c_int32, [c["L"] for c in ch]),
        "d": _arr(C.c_int32, [c["d"] for c in ch]),
        "D": _arr(C.c_int32, [c["D"] for c in ch]),
        "obb": _arr(C.c_int32, [int(c.get("obb", 0)) for c in ch]),
    }
    keep.append(bufs)
    sm = StarModel()
    sm.n_levels = n
    sm.h_el = bufs["h"]
    sm.init_el = bufs["i"]
    sm.n_chains = len(ch)
    sm.coupling = bufs["A"]
    sm.alpha, sm.wc, sm.s = bufs["al"], bufs["wc"], bufs["s"]
    sm.length, sm.local_dim, sm.bond_dim = bufs["L"], bufs["d"], bufs["D"]
    sm.topology = 1 if m["topology"] == "er" else 0
    sm.er_bond_dim = int(m.get("er_D", ch[0]["D"] if ch else 1))
    sm.obb_dim = bufs["obb"]
    sm.potential = 1 if m.get("potential") else 0
    return sm


def tree_struct(parent, phys, bond, ops, terms, init_local, observe=(), keep=None):
    """Marshal a generic tree: ops is a list of square complex matrices,
    terms a list of (coef, node_a, op_a, node_b, op_b) with node_b = -1 for
    on-site terms, init_local a list of per-node amplitude vectors, observe a
    list of (node, op)."""
    t = Tree()
    bufs = {
        "p": _arr(C.c_int32, parent), "d": _arr(C.c_int32, phys), "b": _arr(C.c_int32, bond),
        "od": _arr(C.c_int32, [np.asarray(o).shape[0] for o in ops]),
        "o": _c64_array(np.concatenate([np.asarray(o).reshape(-1) for o in ops]) if ops else [0]),
        "t": (Term * max(len(terms), 1))(*[Term(a, oa, b, ob, c) for (c, a, oa, b, ob) in terms]),
        "i": _c64_array(np.concatenate([np.asarray(x).reshape(-1) for x in init_local])),
        "on": _arr(C.c_int32, [o[0] for o in observe]), "oo": _arr(C.c_int32, [o[1] for o in observe]),
    }
    if keep is not None:
        keep.append(bufs)
    t.n_nodes = len(parent)
    t.parent, t.phys_dim, t.bond_dim = bufs["p"], bufs["d"], bufs["b"]
    t.n_ops, t.op_dim, t.op_data = len(ops), bufs["od"], bufs["o"]
    t.n_terms, t.terms = len(terms), bufs["t"]
    t.init_local = bufs["i"]
    t.n_observe, t.observe_node, t.observe_op = len(observe), bufs["on"], bufs["oo"]
    t._keep = bufs
    return t


class Context:
    """A built TTNS context on cuda:0 (or the given device).

    ``models`` is a list of workload descriptions (star / ER models) or,
    with ``trees=True``, a list of Tree structs from ``tree_struct``.
    """

    def __init__(self, models, opts=None, device="cuda:0", trees=False, stream=None, noalloc=False):
        import torch
        self.torch = torch
        L = lib()
        self.keep = []
        self.opts = opts if opts is not None else default_opts()
        self.n_trees = len(models)
        if noalloc:  # ttns_star_build_noalloc: the library's static workspace
            arr = (StarModel * len(models))(*[star_model(m, self.keep) for m in models])
            self.keep.append(arr)
            self.device = torch.device(device)
            self.ws = None
            with torch.cuda.device(self.device):
                self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
                self.ctx = C.c_void_p()
                check(L.ttns_star_build_noalloc(arr, len(models), C.byref(self.opts),
                                                C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx)))
            return
        if trees:
            arr = (Tree * len(models))(*models)
            size_fn, build_fn = L.ttns_workspace_size, L.ttns_build
        else:
            arr = (StarModel * len(models))(*[star_model(m, self.keep) for m in models])
            size_fn, build_fn = L.ttns_star_workspace_size, L.ttns_star_build
        self.keep.append(arr)
        nbytes = C.c_size_t()
        check(size_fn(arr, len(models), C.byref(self.opts), C.byref(nbytes)))
        self.nbytes = nbytes.value
        self.device = torch.device(device)
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        check(build_fn(arr, len(models), C.byref(self.opts), C.c_void_p(self.ws_ptr),
                       C.c_size_t(self.nbytes), C.c_void_p(self.stream.cuda_stream),
                       C.byref(self.ctx)))
        self.n_trees = len(models)

    def close(self):
        if self.ctx:
            lib().ttns_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls -------------------------------------------------------------
    def ttns_tdvp_step(self, dt, n_steps=1):
        check(lib().ttns_tdvp_step(self.ctx, float(dt), int(n_steps)))

    def ttns_apply_heff(self, tree, node, x_dev, y_dev):
        check(lib().ttns_apply_heff(self.ctx, int(tree), int(node), C.c_void_p(x_dev.data_ptr()),
                                    C.c_void_p(y_dev.data_ptr())))

    def ttns_observe(self, kind, tree=0, index=0, n=None):
        if n is None:
            n = self._obs_size(kind, tree, index)
        out = np.zeros(max(n, 1), dtype=np.float64)
        check(lib().ttns_observe(self.ctx, int(kind), int(tree), int(index),
                                 out.ctypes.data_as(C.POINTER(C.c_double)), C.c_size_t(out.size)))
        return out[:n]

    def _obs_size(self, kind, tree, index):
        if kind == OBS_HISTORY:
            st = self.ttns_observe(OBS_STATS, tree, n=5)
            rs = int(self.ttns_observe(OBS_RECORD_SIZE, tree, n=1)[0])
            return int(st[0]) * rs
        if kind == OBS_STATS:
            return 5
        if kind in (OBS_NORM, OBS_ENERGY, OBS_RECORD_SIZE):
            return 1
        raise ValueError("pass n for this kind")

    # -- conveniences --------------------------------------------------------
    def history(self, tree=0, n_levels=None, n_obs=None):
        """Records as dict of arrays: rdm (K, n, n), norm, energy, local."""
        rs = int(self.ttns_observe(OBS_RECORD_SIZE, tree, n=1)[0])
        h = self.ttns_observe(OBS_HISTORY, tree).reshape(-1, rs)
        if n_levels is None:
            n_levels = int(round(np.sqrt((rs - 2) / 2)))
            while 2 * n_levels * n_levels + 2 > rs:
                n_levels -= 1
        nn = 2 * n_levels * n_levels
        rdm = h[:, :nn].reshape(-1, n_levels, n_levels, 2)
        return {"rdm": rdm[..., 0] + 1j * rdm[..., 1], "norm": h[:, nn], "energy": h[:, nn + 1],
                "local": h[:, nn + 2:]}

    def tensor(self, tree, node, shape):
        flat = self.ttns_observe(OBS_TENSOR, tree, node, n=2 * int(np.prod(shape)))
        return (flat[0::2] + 1j * flat[1::2]).reshape(shape)

    def stats(self, tree=0):
        s = self.ttns_observe(OBS_STATS, tree, n=5)
        return {"records": int(s[0]), "guarded": int(s[1]), "steps": int(s[2]),
                "breakdowns": int(s[3]), "flags": int(s[4])}

    def step_flops(self, tree=0):
        """Algorithmic flops of one step of ``tree``: (total, H_eff part)."""
        f = self.ttns_observe(OBS_STEP_FLOPS, tree, n=2)
        return float(f[0]), float(f[1])

    def entropy(self, tree, node):
        """Entanglement entropy across the bond (node, parent(node))."""
        return float(self.ttns_observe(OBS_ENTROPY, tree, node, n=1)[0])

    def energy_surfaces(self, tree=0, rank_tol=1e-5, matrix=False):
        """Eigenvalues (ascending) of the effective matrix of this context's
        operator between (bath Schmidt state, electronic state) products;
        with matrix=True also the matrix ((r n) x (r n) complex)."""
        n = int(round(np.sqrt((int(self.ttns_observe(OBS_RECORD_SIZE, tree, n=1)[0]) - 2) / 2)))
        while 2 * n * n + 2 > int(self.ttns_observe(OBS_RECORD_SIZE, tree, n=1)[0]):
            n -= 1
        vals = np.zeros(n * n)
        mat = np.zeros(2 * n ** 4) if matrix else None
        r = C.c_int32()
        check(lib().ttns_energy_surfaces(self.ctx, int(tree), float(rank_tol), C.byref(r),
                                         vals.ctypes.data_as(C.POINTER(C.c_double)),
                                         mat.ctypes.data_as(C.POINTER(C.c_double)) if matrix else None,
                                         C.c_size_t(vals.size)))
        N = r.value * n
        if not matrix:
            return vals[:N]
        M = mat[:2 * N * N].reshape(N, N, 2)
        return vals[:N], M[..., 0] + 1j * M[..., 1]

    def copy_state_from(self, src, tree=0, src_tree=0):
        """This context's tree takes src's state (ttns_copy_state)."""
        check(lib().ttns_copy_state(self.ctx, int(tree), src.ctx, int(src_tree)))

    def bond_dims(self, tree, n_nodes):
        return self.ttns_observe(OBS_BOND_DIMS, tree, n=n_nodes).astype(int)

    def tuning_report(self):
        """The autotuner's measurements and choices (empty without
        TTNS_FLAG_AUTOTUNE)."""
        need = C.c_size_t()
        check(lib().ttns_tuning_report(self.ctx, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        check(lib().ttns_tuning_report(self.ctx, buf, need.value, None))
        return buf.value.decode()

    def profile(self, enable=True):
        check(lib().ttns_profile(self.ctx, 1 if enable else 0))

    def profile_kernels(self):
        """Per kernel id: total ms, launches, algorithmic flops and bytes."""
        out = {}
        for kid, name in KERNELS.items():
            ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
            check(lib().ttns_profile_kernel(self.ctx, kid, C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)))
            if n.value:
                out[kid] = {"name": name, "ms": ms.value, "launches": n.value, "flops": fl.value,
                            "bytes": by.value}
        return out

    def profile_read(self, reset=True):
        ms, n, fl = C.c_double(), C.c_int64(), C.c_double()
        check(lib().ttns_profile_read(self.ctx, 1 if reset else 0, C.byref(ms), C.byref(n), C.byref(fl)))
        return {"avg_ms": ms.value, "launches": n.value, "flops_per_launch": fl.value}

"""Host-side checks of the C-ABI (no device work): the library loads and
exports every symbol that include/*.h declares, the model-assembly step (chain
mapping) matches the oracle, and invalid inputs are rejected before any
device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle.chain import ohmic_chain
from paper_1710_01362_amd import ttns as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    from paper_1710_01362_amd import ttnn as N
    declared = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            hdr = open(os.path.join(ROOT, "include", h)).read()
            declared |= set(re.findall(r"\b(ttn[sn]_[a-z_]+)\s*\(", hdr))
    assert declared == set(T.EXPORTED) | set(N.EXPORTED)
    L = T.lib()
    N.lib()
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("alpha,wc,s,L", [(0.1, 1.0, 1.0, 10), (0.2, 0.2, 1.0, 40), (0.05, 2.0, 0.5, 7), (0.3, 1.0, 1.0, 1)])
def test_chain_mapping_matches_oracle(alpha, wc, s, L):
    c0, eps, hop = T.ttns_ohmic_chain(alpha, wc, s, L)
    c0o, epso, hopo = ohmic_chain(alpha, wc, s, L)
    assert abs(c0 - c0o) <= 1e-15 * wc
    np.testing.assert_allclose(eps, epso, rtol=0, atol=1e-15 * wc)
    np.testing.assert_allclose(hop, hopo, rtol=0, atol=1e-15 * wc)


def _ws_size(models, **kw):
    keep = []
    arr = (T.StarModel * len(models))(*[T.star_model(m, keep) for m in models])
    nb = C.c_size_t()
    o = T.default_opts(**kw)
    rc = T.lib().ttns_star_workspace_size(arr, len(models), C.byref(o), C.byref(nb))
    return rc, nb.value


@pytest.mark.parametrize("model", [W.spin_boson_reference(), W.vibronic_reference(), W.large_tree(),
                                   W.vibronic_small(), dict(W.vibronic_small(), topology="er")],
                         ids=["spin_boson", "vibronic", "large_er", "vibronic_small", "small_er"])
def test_programs_plan_and_pass_range_checks(model):
    """Planning every op of the init and step programs, with the host range
    checker over each descriptor, succeeds for every workload."""
    rc, nbytes = _ws_size([model], record_capacity=model["steps"] + 1)
    assert rc == T.TTNS_OK, T.lib().ttns_last_error(None)
    assert nbytes > 0


@pytest.mark.parametrize("model", [
    W.vibronic(seed=2, n_levels=5, n_chains=2, L=4, d=4, D=4, steps=4),   # levels > bond dims
    W.spin_boson(L=1, d=1, D=1, delta=0.6, steps=5),
    W.spin_boson(L=3, d=3, D=1, delta=0.4, alpha=0.2, steps=6),
    W.vibronic(seed=4, n_chains=8, L=3, d=4, D=6, steps=4, topology="er", er_D=6),
], ids=["levels_gt_D", "trivial_bath", "bond_dim_1", "er8_small"])
def test_edge_configurations_plan(model):
    rc, nbytes = _ws_size([model], record_capacity=model["steps"] + 1)
    assert rc == T.TTNS_OK, T.lib().ttns_last_error(None)


def test_batched_ensemble_plans():
    rc, nbytes = _ws_size(W.ensemble(n=16), record_capacity=101)
    assert rc == T.TTNS_OK, T.lib().ttns_last_error(None)


def _tree(parent, phys, bond, ops, terms, init, observe=()):
    keep = []
    return T.tree_struct(parent, phys, bond, ops, terms, init, observe, keep), keep


def _build_status(tree, ws_bytes=1 << 20, **kw):
    ctx = C.c_void_p()
    o = T.default_opts(**kw)
    return T.lib().ttns_build(C.byref(tree), 1, C.byref(o), C.c_void_p(4096), C.c_size_t(ws_bytes),
                              None, C.byref(ctx))


def _spin_chain(coef_hop=0.3, coef_back=0.3, parent=(-1, 0, 1)):
    sz = np.diag([1.0, -1.0]).astype(complex)
    b = np.array([[0, 1], [0, 0]], dtype=complex)
    ops = [sz, b, b.T.copy()]
    terms = [(0.5, 0, 0, -1, -1), (coef_hop, 1, 2, 2, 1), (coef_back, 1, 1, 2, 2), (0.2, 0, 0, 1, 1),
             (0.2, 0, 0, 1, 2)]
    init = [np.array([1, 0]), np.array([1, 0]), np.array([1, 0])]
    return _tree(list(parent), [2, 2, 2], [0, 2, 2], ops, terms, init)


def test_rejects_non_hermitian_operator_sum():
    t, keep = _spin_chain(coef_back=0.1)
    assert _build_status(t) == T.TTNS_EINVAL
    assert b"Hermitian" in T.lib().ttns_last_error(None)


def test_rejects_bad_topology():
    t, keep = _spin_chain(parent=(-1, 2, 0))
    assert _build_status(t) == T.TTNS_EINVAL


def test_rejects_non_finite_input():
    t, keep = _spin_chain(coef_hop=float("nan"), coef_back=float("nan"))
    assert _build_status(t) == T.TTNS_ENUMERIC


def test_reports_small_workspace():
    t, keep = _spin_chain()
    assert _build_status(t, ws_bytes=1024) == T.TTNS_ENOMEM
    assert b"too small" in T.lib().ttns_last_error(None)


def test_rejects_bad_options():
    t, keep = _spin_chain()
    assert _build_status(t, krylov_dim=0) == T.TTNS_EINVAL
    assert _build_status(t, krylov_dim=17) == T.TTNS_EINVAL
    assert _build_status(t, record_capacity=0) == T.TTNS_EINVAL
    assert _build_status(t, flags=4) == T.TTNS_EINVAL
    assert b"flags" in T.lib().ttns_last_error(None)
    assert _build_status(t, executor=3) == T.TTNS_EINVAL
    assert b"executor" in T.lib().ttns_last_error(None)


@pytest.mark.parametrize("model", [W.vibronic_reference(), W.large_tree(), W.vibronic_small()],
                         ids=["vibronic", "large_er", "vibronic_small"])
def test_autotune_probe_plan_bounds_the_workspace(model):
    """With TTNS_FLAG_AUTOTUNE the size query plans every candidate (the
    probe build); any final plan the autotuner picks needs no more."""
    rc0, plain = _ws_size([model], record_capacity=2)
    rc1, tuned = _ws_size([model], record_capacity=2, flags=T.TTNS_FLAG_AUTOTUNE)
    rc2, all_mfma = _ws_size([model], record_capacity=2, flags=T.TTNS_FLAG_MFMA_ALL)
    assert rc0 == rc1 == rc2 == T.TTNS_OK
    assert tuned >= plain and tuned >= all_mfma


def test_overflowing_but_finite_hamiltonian_is_accepted_by_the_size_query():
    """The run-time numerical check (ttns_observe -> TTNS_ENUMERIC) is tested
    with a Hamiltonian of scale 1e300: finite, so validation accepts it."""
    rc, nbytes = _ws_size([W.spin_boson(L=3, d=3, D=2, delta=1e300, steps=2)], record_capacity=4)
    assert rc == T.TTNS_OK and nbytes > 0


def test_noalloc_build_rejects_trees_beyond_the_static_workspace():
    """The allocation-free build checks the size before any device call:
    the five-level tree needs more than the 64 MiB static array."""
    import ctypes as C
    keep = []
    arr = (T.StarModel * 1)(T.star_model(W.vibronic_reference(), keep))
    ctx = C.c_void_p()
    o = T.default_opts(record_capacity=2)
    rc = T.lib().ttns_star_build_noalloc(arr, 1, C.byref(o), None, C.byref(ctx))
    assert rc == T.TTNS_ENOMEM and not ctx.value
    assert b"static workspace holds 67108864" in T.lib().ttns_last_error(None)
    o = T.default_opts(record_capacity=2, flags=T.TTNS_FLAG_AUTOTUNE)
    arr = (T.StarModel * 1)(T.star_model(W.spin_boson_reference(), keep))
    assert T.lib().ttns_star_build_noalloc(arr, 1, C.byref(o), None, C.byref(ctx)) == T.TTNS_EINVAL


def test_binding_refuses_a_library_with_other_struct_layouts():
    """The binding compares its ctypes struct sizes with the library's at
    load time; a stale library (built from other headers) is refused with a
    message instead of reading the arguments wrongly."""
    T.lib()  # the in-tree build matches

    class Fake:
        @staticmethod
        def ttns_struct_sizes(out, n):
            for i in range(n):
                out[i] = 1
            return T.TTNS_OK
    with pytest.raises(RuntimeError, match="other headers"):
        T._check_struct_sizes(Fake())

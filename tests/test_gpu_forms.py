"""GPU tests of the matrix-core H_eff path and the reduced-precision forms.

* FP64 on the matrix cores (large nodes): H_eff equals the oracle's to
  1e-12 relative at t = 0 (exact gauges) -- the same bar as the scalar path.
* FP32 and split-BF16 (bf16x3) H_eff contractions: every operand is rounded
  once (FP32: 2^-24 relative; bf16x3: hi + lo carries 16 mantissa bits and
  the dropped lo*lo term is ~2^-32) and products are accumulated in FP32
  over K = 2D terms, so the elementwise error is bounded by ~K * 2^-24 of the
  row norm; we hold it to 2e-5 relative to the largest entry.
  (Small trees: every node is put on the matrix cores with
  TTNS_FLAG_MFMA_ALL; by default only nodes of >= 16384 entries are.)
* Whole trajectories with the reduced-precision contractions (Lanczos,
  exponentials, QR and environments stay FP64): population error against the
  FP64 oracle within 1e-5 (stated tolerance of the precision forms).
"""
import numpy as np
import pytest

import workloads as W
from oracle.model import build_tree
from oracle.ttns import TTNS, run

pytestmark = pytest.mark.gpu


def _T():
    from paper_1710_01362_amd import ttns as T
    return T


def _apply_vs_oracle(m, precision, nodes, rel):
    import torch
    T = _T()
    ctx = T.Context([m], opts=T.default_opts(record_capacity=2, precision=precision,
                                             executor=T.TTNS_EXEC_WIDE,
                                             flags=T.TTNS_FLAG_MFMA_ALL))
    tt = TTNS(build_tree(m))
    rng = np.random.default_rng(11)
    worst = 0.0
    for v in nodes:
        shp = tt.shape[v]
        X = rng.normal(size=shp) + 1j * rng.normal(size=shp)
        xd = torch.from_numpy(X.reshape(-1).copy()).to("cuda")
        yd = torch.zeros_like(xd)
        ctx.ttns_apply_heff(0, v, xd, yd)
        got = yd.cpu().numpy().reshape(shp)
        tt.move_to(v)
        ref = tt.apply_heff(v, X)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        assert err <= rel, (v, err)
    ctx.close()
    return worst


def test_fp64_matrix_cores_root_of_reference_tree():
    """The 5 x 20^4 root of the five-level tree runs on FP64 MFMA tiles."""
    m = W.vibronic_reference()
    _apply_vs_oracle(m, 0, [0], 1e-12)


@pytest.mark.parametrize("precision", [1, 2], ids=["fp32", "bf16x3"])
def test_reduced_precision_root_of_reference_tree(precision):
    """The 5 x 20^4 root on 64-column tiles (small trees use 16-column ones)."""
    m = W.vibronic_reference()
    _apply_vs_oracle(m, precision, [0], 2e-5)


@pytest.mark.parametrize("precision", [1, 2], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("topology", ["star", "er"])
def test_reduced_precision_apply(precision, topology):
    m = dict(W.vibronic(seed=5, n_chains=4, L=5, d=6, D=6, steps=2), topology=topology)
    tt = TTNS(build_tree(m))
    nodes = sorted(set([0, 1, 2, tt.n - 1] + [v for v in range(tt.n) if tt.phys[v] == 1][:2]))
    _apply_vs_oracle(m, precision, nodes, 2e-5)


@pytest.mark.parametrize("precision", [1, 2], ids=["fp32", "bf16x3"])
def test_reduced_precision_trajectory_population_error(precision):
    T = _T()
    m = W.vibronic(seed=2, n_chains=4, L=8, d=8, D=8, steps=20)
    ctx = T.Context([m], opts=T.default_opts(record_capacity=m["steps"] + 1, precision=precision,
                                             flags=T.TTNS_FLAG_MFMA_ALL))
    ctx.ttns_tdvp_step(m["dt"], m["steps"])
    hg = ctx.history()
    ctx.close()
    _, ho = run(m)
    pop = np.abs(np.einsum("kjj->kj", hg["rdm"]).real - np.einsum("kjj->kj", ho["rdm"]).real).max()
    assert pop <= 1e-5, pop
    # the FP64 parts still conserve the norm to round-off of the reduced products
    assert np.abs(hg["norm"] - 1).max() <= 1e-5


def test_large_er_tree_full_size():
    """The large tree at its full size (5-level root, 6 ER nodes, 8 chains x
    100 sites, d = 30, D = 48), in the wide executor as the benchmark runs it:

    * FP64 H_eff at sampled nodes (root, ER nodes, a chain head, a chain
      site, a chain end) against the oracle at t = 0: 1e-12 relative;
    * the split-BF16 form at the same nodes: 2e-5 relative;
    * one TDVP step in both precisions: the split-BF16 populations within
      1e-5 of the FP64 GPU run, FP64 norm and energy conserved to 1e-10.
    """
    import torch
    T = _T()
    m = W.large_tree()
    tt = TTNS(build_tree(m))
    nodes = [0, 1, 2, 3, 4, 102, 103]
    rng = np.random.default_rng(13)
    inputs = {v: rng.normal(size=tt.shape[v]) + 1j * rng.normal(size=tt.shape[v]) for v in nodes}
    refs = {}
    for v in nodes:
        tt.move_to(v)
        refs[v] = tt.apply_heff(v, inputs[v])
    hist = {}
    for prec, rel in ((0, 1e-12), (2, 2e-5)):
        ctx = T.Context([m], opts=T.default_opts(record_capacity=3, precision=prec, executor=T.TTNS_EXEC_WIDE))
        for v in nodes:
            xd = torch.from_numpy(inputs[v].reshape(-1).copy()).to("cuda")
            yd = torch.zeros_like(xd)
            ctx.ttns_apply_heff(0, v, xd, yd)
            got = yd.cpu().numpy().reshape(tt.shape[v])
            err = np.abs(got - refs[v]).max() / np.abs(refs[v]).max()
            assert err <= rel, (prec, v, err)
        ctx.ttns_tdvp_step(m["dt"], 1)
        hist[prec] = ctx.history()
        ctx.close()
    h64, h16 = hist[0], hist[2]
    assert np.abs(h64["norm"] - 1).max() <= 1e-10
    assert np.abs(h64["energy"] - h64["energy"][0]).max() <= 1e-10 * max(1.0, abs(h64["energy"][0]))
    pop = np.abs(np.einsum("kjj->kj", h16["rdm"]).real - np.einsum("kjj->kj", h64["rdm"]).real).max()
    assert pop <= 1e-5, pop


@pytest.mark.parametrize("precision", [1, 2], ids=["fp32", "bf16x3"])
def test_reduced_precision_in_the_persistent_batch(precision):
    """The batched (one workgroup per tree) executor runs the reduced-precision
    forms on the matrix cores too: an uneven batch of ensemble-recipe
    instances in one persistent launch per step, each within 1e-5 in
    populations of its FP64 oracle run, and visibly not the FP64 result
    (the form is really used)."""
    T = _T()
    models = []
    for m in W.ensemble(n=6):
        m = dict(m)
        m["chains"] = [dict(m["chains"][0], L=min(m["chains"][0]["L"], 12))]
        m["steps"] = 12
        models.append(m)
    opts = dict(record_capacity=13, executor=T.TTNS_EXEC_PERSISTENT)
    ctx = T.Context(models, opts=T.default_opts(precision=precision, **opts))
    ctx.ttns_tdvp_step(models[0]["dt"], 12)
    hs = [ctx.history(i) for i in range(len(models))]
    ctx.close()
    ctx = T.Context(models, opts=T.default_opts(**opts))
    ctx.ttns_tdvp_step(models[0]["dt"], 12)
    h64 = [ctx.history(i) for i in range(len(models))]
    ctx.close()
    worst, diff = 0.0, 0.0
    for m, hg, hf in zip(models, hs, h64):
        _, ho = run(m)
        pg = np.einsum("kjj->kj", hg["rdm"]).real
        po = np.einsum("kjj->kj", ho["rdm"]).real
        worst = max(worst, np.abs(pg - po).max())
        diff = max(diff, np.abs(hg["rdm"] - hf["rdm"]).max())
        assert np.abs(hg["norm"] - 1).max() <= 1e-5
    print("persistent batch, precision %d: population error vs oracle %.2e, vs FP64 GPU %.2e" % (precision, worst, diff))
    assert worst <= 1e-5, worst
    assert diff > 1e-13  # the contractions did run in reduced precision

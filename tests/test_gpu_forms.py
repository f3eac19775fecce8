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

"""The allocation-free build (ttns_star_build_noalloc): a context in the
library's static per-device workspace gives the same trajectory as one in a
caller workspace, on two builds in a row (the second smaller, so it runs on
what the first left in the array), and refuses a second live context on the
same device."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _T():
    from paper_1710_01362_amd import ttns as T
    return T


def _history(models, steps, noalloc):
    T = _T()
    ctx = T.Context(models, opts=T.default_opts(record_capacity=steps + 1), noalloc=noalloc)
    ctx.ttns_tdvp_step(models[0]["dt"], steps)
    hs = [ctx.history(i) for i in range(len(models))]
    st = ctx.stats(0)
    ctx.close()
    return hs, st


def test_noalloc_build_matches_workspace_build_twice():
    cases = [([W.spin_boson_reference()], 40),
             ([W.spin_boson(L=5, d=4, D=3, delta=0.5, alpha=0.2, steps=10)], 10)]
    for models, steps in cases:
        ref, _ = _history(models, steps, False)
        got, st = _history(models, steps, True)
        assert st["steps"] == steps
        for hr, hg in zip(ref, got):
            for k in ("rdm", "norm", "energy", "local"):
                assert hg[k].shape == hr[k].shape
                assert np.abs(hg[k] - hr[k]).max() <= 1e-12, k


def test_noalloc_batch_of_trees():
    """Several trees (the persistent executor) in the static workspace."""
    models = [W.spin_boson(L=4, d=4, D=3, delta=0.3, alpha=0.05, steps=6),
              W.spin_boson(L=7, d=5, D=4, delta=0.8, alpha=0.25, steps=6)]
    ref, _ = _history(models, 6, False)
    got, _ = _history(models, 6, True)
    for hr, hg in zip(ref, got):
        assert np.abs(hg["rdm"] - hr["rdm"]).max() <= 1e-12


def test_noalloc_workspace_held_by_one_context():
    T = _T()
    m = W.spin_boson(L=4, d=4, D=3, steps=2)
    a = T.Context([m], opts=T.default_opts(record_capacity=3), noalloc=True)
    with pytest.raises(T.TTNSError) as err:
        T.Context([m], opts=T.default_opts(record_capacity=3), noalloc=True)
    assert err.value.code == T.TTNS_EINVAL
    a.close()
    b = T.Context([m], opts=T.default_opts(record_capacity=3), noalloc=True)
    b.ttns_tdvp_step(m["dt"], 2)
    assert b.stats()["steps"] == 2
    b.close()

"""Host-side checks of the learned-propagator C-ABI (include/ttnn.h): sizes
and parameter layout agree with the oracle's network, the conditioning
vector of a star model matches the oracle's, and invalid configurations are
rejected without any device call."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from oracle import learned as OL
from paper_1710_01362_amd import ttnn as N
from paper_1710_01362_amd import ttns as T


@pytest.mark.parametrize("skip", [0, 1])
@pytest.mark.parametrize("n,window,nc,hidden,layers", [(5, 40, 39, 512, 3), (2, 3, 0, 7, 1), (3, 4, 5, 16, 2)])
def test_param_count_matches_oracle_layout(n, window, nc, hidden, layers, skip):
    cfg = N.config(n, window, nc, hidden, layers, 64, skip)
    sizes = OL.layer_sizes(window, n * n, nc, hidden, layers, bool(skip))
    params = OL.init_params(sizes, np.random.default_rng(0), bool(skip))
    assert N.param_count(cfg) == OL.flatten(params).size
    assert N.workspace_size(cfg) >= 4 * (4 * N.param_count(cfg) + 64 * (window * n * n + nc))


def test_conditioning_matches_oracle():
    for m in (W.vibronic_reference(), W.vibronic_small(), W.vibronic(seed=9, n_levels=3, n_chains=2)):
        got = N.conditioning(m)
        ref = OL.conditioning(m)
        assert got.shape == ref.shape
        np.testing.assert_array_equal(got, ref.astype(np.float32))
    assert N.conditioning(W.vibronic_reference()).size == 39


@pytest.mark.parametrize("bad", [dict(n_levels=0), dict(n_levels=9), dict(window=0), dict(hidden=0),
                                 dict(layers=0), dict(layers=9), dict(max_batch=0), dict(n_cond=-1),
                                 dict(skip=2)])
def test_bad_configs_rejected(bad):
    kw = dict(n_levels=5, window=4, n_cond=3, hidden=8, layers=2, max_batch=4)
    kw.update(bad)
    cfg = N.config(**kw)
    n = C.c_int64()
    assert N.lib().ttnn_param_count(C.byref(cfg), C.byref(n)) == T.TTNS_EINVAL
    assert T.lib().ttns_last_error(None).decode().startswith("ttnn")


def test_conditioning_output_too_small():
    keep = []
    sm = T.star_model(W.vibronic_reference(), keep)
    out = np.zeros(38, dtype=np.float32)
    n = C.c_int32()
    assert N.lib().ttnn_conditioning(C.byref(sm), out.ctypes.data, 38, C.byref(n)) == T.TTNS_EINVAL


def test_free_propagator_matches_oracle():
    """exp(-i H_S dt) of the library (host FP64, rounded to FP32) against
    the oracle's scipy expm, for the five-level family and a spin."""
    for m, dt in ((W.vibronic_reference(), W.vibronic_reference()["dt"]), (W.spin_boson_reference(), 0.05),
                  (W.vibronic(seed=11, n_levels=3), 7.3)):
        got = N.propagator(m, dt)
        n = int(np.asarray(m["h_el"]).shape[0])
        U = got[0::2].reshape(n, n) + 1j * got[1::2].reshape(n, n)
        ref = OL.propagator(m, dt)
        assert np.abs(U - ref).max() <= 2e-7

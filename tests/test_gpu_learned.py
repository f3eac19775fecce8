"""GPU tests of the learned RDM propagator (include/ttnn.h) against the
FP64 oracle (oracle/learned.py), and of the learned form end to end.

Tolerances.  The library stores parameters and activations in FP32 and
multiplies on FP32 matrix cores with FP32 accumulation; the oracle runs the
same network in FP64 on the same (FP32-representable) parameters and data.
A length-K FP32 dot product carries a rounding error of at most about
K * 2^-24 times the sum of |products|; with K <= 1039 here and sums of
|products| within a small factor of the result, elementwise errors stay
below ~1e-4 of the largest entry of each array, which is the bar used for
losses, gradients and one-step outputs.  Rollouts compound this over their
steps; 20 steps are held to 1e-4 absolute on entries of size <= 1.
Trace distances are computed in FP64 from FP32 inputs: 1e-6 absolute.
"""
import time

import numpy as np
import pytest

import workloads as W
from oracle import learned as OL

pytestmark = pytest.mark.gpu


def _N():
    from paper_1710_01362_amd import ttnn as N
    return N


def _rand_rho(rng, n, k):
    A = rng.normal(size=(k, n, n)) + 1j * rng.normal(size=(k, n, n))
    rho = A @ np.conj(np.swapaxes(A, 1, 2))
    return rho / np.trace(rho, axis1=1, axis2=2).real[:, None, None]


def _setup(n=5, window=4, nc=39, hidden=64, layers=3, S=6, T=30, max_batch=64, seed=0, skip=False):
    """FP32-representable parameters and data shared by both sides."""
    rng = np.random.default_rng(seed)
    sizes = OL.layer_sizes(window, n * n, nc, hidden, layers, skip)
    params = OL.init_params(sizes, rng, skip)
    params = [(Wm, None if b is None else rng.normal(size=b.shape) * 0.05) for Wm, b in params]
    if skip:
        params[-1] = (rng.normal(size=params[-1][0].shape) * 0.01, None)
    flat = OL.flatten(params).astype(np.float32)
    # smooth synthetic RDM trajectories: rho(t) = U(t) rho0 U(t)^dagger
    traj = np.zeros((S, T, n * n))
    for s in range(S):
        rho0 = _rand_rho(rng, n, 1)[0]
        H = rng.normal(size=(n, n))
        H = (H + H.T) / 2
        ev, V = np.linalg.eigh(H)
        for t in range(T):
            U = (V * np.exp(-1j * 0.1 * t * ev)) @ V.T
            traj[s, t] = OL.encode(U @ rho0 @ np.conj(U.T))
    traj = traj.astype(np.float32)
    cond = rng.normal(size=(S, nc)).astype(np.float32)
    # FP32-representable unitaries (as the library's propagators are)
    props = []
    for s in range(S):
        H = rng.normal(size=(n, n)) * 0.3
        U = OL.propagator({"h_el": (H + H.T) / 2}, 1.0)
        props.append(np.stack([U.real, U.imag], axis=-1).reshape(-1).astype(np.float32))
    props = np.stack(props)
    return dict(n=n, window=window, nc=nc, hidden=hidden, layers=layers, sizes=sizes, flat=flat, traj=traj,
                cond=cond, props=props, max_batch=max_batch, rng=rng, skip=skip)


def _unitaries(props, n):
    p = props.astype(np.float64)
    return p[:, 0::2].reshape(-1, n, n) + 1j * p[:, 1::2].reshape(-1, n, n)


def _net(d, propagated=False):
    import torch
    N = _N()
    cfg = N.config(d["n"], d["window"], d["nc"], d["hidden"], d["layers"], d["max_batch"], d["skip"])
    net = N.Net(cfg, d["flat"])
    tr = torch.from_numpy(d["traj"]).to("cuda")
    cd = torch.from_numpy(d["cond"]).to("cuda")
    pr = torch.from_numpy(d["props"]).to("cuda") if propagated else None
    net.ttnn_set_data(tr, cd, pr)
    return net, tr, cd


def _samples(d, B):
    rng = d["rng"]
    S, T = d["traj"].shape[:2]
    return np.stack([rng.integers(0, S, B), rng.integers(d["window"] - 1, T - 1, B)], axis=1).astype(np.int32)


def _oracle_params(d):
    return OL.unflatten(d["flat"].astype(np.float64), d["sizes"], d["skip"])


def test_parameters_round_trip():
    d = _setup()
    net, _, _ = _net(d)
    np.testing.assert_array_equal(net.ttnn_get_params(), d["flat"])
    net.close()


VARIANTS = [(False, False), (True, False), (True, True)]
VARIANT_IDS = ["plain", "propagated", "propagated-skip"]


@pytest.mark.parametrize("propagated,skip", VARIANTS, ids=VARIANT_IDS)
def test_loss_and_gradients_match_oracle(propagated, skip):
    d = _setup(skip=skip)
    net, _, _ = _net(d, propagated)
    U = _unitaries(d["props"], d["n"]) if propagated else None
    for B in (1, 37, 64):  # one row, a ragged tile, a full batch
        smp = _samples(d, B)
        loss, grad = net.ttnn_gradients(smp)
        X, Y, R = OL.windows(d["traj"].astype(np.float64), d["cond"].astype(np.float64), smp, d["window"], U,
                             d["n"], skip)
        lo, go = OL.loss_and_grads(_oracle_params(d), X, Y, d["n"] ** 2, d["window"], R)
        assert abs(loss - lo) <= 1e-4 * lo, (B, loss, lo)
        gref = OL.flatten(go)
        # per parameter block (W and b of each layer, then the skip matrix)
        blocks = [s for a, b in zip(d["sizes"][:-1], d["sizes"][1:]) for s in (a * b, b)]
        if skip:
            blocks.append(d["sizes"][0] * d["sizes"][-1])
        off = 0
        for size in blocks:
            blk, ref = grad[off:off + size], gref[off:off + size]
            err = np.abs(blk - ref).max() / np.abs(ref).max()
            assert err <= 1e-4, (B, off, err)
            off += size
    net.close()


def test_adam_step_matches_oracle():
    d = _setup(seed=1, skip=True)
    net, _, _ = _net(d)
    smp = _samples(d, 48)
    lr = 1e-3
    X, Y, R = OL.windows(d["traj"].astype(np.float64), d["cond"].astype(np.float64), smp, d["window"], skip=True)
    p = _oracle_params(d)
    m = [(np.zeros_like(Wm), None if b is None else np.zeros_like(b)) for Wm, b in p]
    v = [(np.zeros_like(Wm), None if b is None else np.zeros_like(b)) for Wm, b in p]
    for t in (1, 2, 3):
        net.ttnn_train_step(smp, lr)
        _, g = OL.loss_and_grads(p, X, Y, d["n"] ** 2, d["window"], R)
        p, m, v = OL.adam_step(p, g, m, v, t, lr)
    got = net.ttnn_get_params().astype(np.float64)
    ref = OL.flatten(p)
    gflat = np.abs(OL.flatten(g))
    # Adam moves each parameter by about lr * sign(g): compare the moves where
    # the gradient is well above FP32 noise, and bound all of them
    move_ref = ref - d["flat"]
    move_got = got - d["flat"]
    # gradients carry ~1e-4 max|g| of FP32 rounding: an element of size
    # >= 3e-2 max|g| moves its Adam ratio by <~1e-2
    big = gflat > 3e-2 * gflat.max()
    assert np.abs(move_got[big] - move_ref[big]).max() <= 2e-2 * lr
    assert np.abs(move_got - move_ref).max() <= 6 * lr
    net.close()


@pytest.mark.parametrize("propagated,skip", VARIANTS, ids=VARIANT_IDS)
def test_rollout_matches_oracle(propagated, skip):
    import torch
    d = _setup(seed=2, max_batch=16, skip=skip)
    # a contractive network (small output layer): an untrained random map
    # would amplify rounding differences over the rollout
    p = _oracle_params(d)
    k = -2 if skip else -1
    p[k] = (0.05 * p[k][0], np.zeros_like(p[k][1]))
    if skip:
        p[-1] = (0.1 * p[-1][0], None)
    d["flat"] = OL.flatten(p).astype(np.float32)
    net, _, _ = _net(d)
    B, steps = 9, 20
    S = d["traj"].shape[0]
    init = np.stack([d["traj"][b % S, 2 * b:2 * b + d["window"]] for b in range(B)])  # windows from the data
    cond = np.stack([d["cond"][b % S] for b in range(B)])
    props = np.stack([d["props"][b % S] for b in range(B)])
    pd = torch.from_numpy(props).to("cuda") if propagated else None
    out = net.ttnn_rollout(torch.from_numpy(init).to("cuda"), torch.from_numpy(cond).to("cuda"), steps, pd)
    got = out.cpu().numpy()
    ref = OL.rollout(_oracle_params(d), init.astype(np.float64), cond.astype(np.float64), steps, d["n"],
                     d["window"], _unitaries(props, d["n"]) if propagated else None)
    assert np.abs(got - ref).max() <= 1e-4
    # unit trace after every step
    assert np.abs(got[..., :d["n"]].sum(-1) - 1).max() <= 1e-5
    net.close()


def test_encode_trace_distance_judge_select():
    import torch
    d = _setup(seed=3, max_batch=8)
    net, _, _ = _net(d)
    rng = np.random.default_rng(4)
    B, S, n = 7, 11, d["n"]
    rho = _rand_rho(rng, n, B * S).reshape(B, S, n, n)
    sig = rho + 1e-3 * rng.uniform(0, 1, size=(B, 1, 1, 1)) * (_rand_rho(rng, n, B * S).reshape(B, S, n, n) - rho)
    e_rho = net.ttnn_encode(torch.from_numpy(rho).to("cuda"))
    e_sig = net.ttnn_encode(torch.from_numpy(sig).to("cuda"))
    np.testing.assert_array_equal(e_rho.cpu().numpy(), OL.encode(rho).astype(np.float32))
    tol = 5e-4
    dist, worst, accept = net.ttnn_judge(e_rho, e_sig, tol)
    # oracle distances of the same FP32 encodings
    dref = OL.trace_distance(OL.decode(e_rho.cpu().numpy().astype(np.float64), n),
                             OL.decode(e_sig.cpu().numpy().astype(np.float64), n))
    assert np.abs(dist.cpu().numpy() - dref).max() <= 1e-6
    wref = dref.max(axis=1)
    np.testing.assert_allclose(worst.cpu().numpy(), wref, atol=1e-6)
    clear = np.abs(wref - tol) > 1e-6
    assert (accept.cpu().numpy()[clear] == (wref[clear] <= tol)).all()
    sel = net.ttnn_select(e_rho, e_sig, accept).cpu().numpy()
    a = accept.cpu().numpy().astype(bool)
    np.testing.assert_array_equal(sel[a], e_rho.cpu().numpy()[a])
    np.testing.assert_array_equal(sel[~a], e_sig.cpu().numpy()[~a])
    net.close()


def test_bad_samples_rejected_before_launch():
    from paper_1710_01362_amd import ttns as T
    d = _setup(seed=5)
    net, _, _ = _net(d)
    T_ = d["traj"].shape[1]
    for bad in ([[0, d["window"] - 2]], [[0, T_ - 1]], [[6, 5]], [[-1, 5]]):
        with pytest.raises(T.TTNSError) as e:
            net.ttnn_gradients(np.array(bad, dtype=np.int32))
        assert e.value.code == T.TTNS_EINVAL
    with pytest.raises(T.TTNSError):
        net.ttnn_gradients(_samples(d, d["max_batch"] + 1))
    net.close()


# ------------------------------------------------------------- end to end
def _ttns_trajectories(models, steps):
    """RDM trajectories (sets, steps + 1, n, n) of the TTNS-TDVP GPU library,
    all sets in one persistent launch per step; also the wall time."""
    import torch
    from paper_1710_01362_amd import ttns as T
    ctx = T.Context(models, opts=T.default_opts(record_capacity=steps + 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.ttns_tdvp_step(models[0]["dt"], steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rdm = np.stack([ctx.history(k)["rdm"] for k in range(len(models))])
    ctx.close()
    return rdm, el


def test_learned_form_trains_on_ttns_data_and_is_judged_by_it():
    """Train on TTNS RDM trajectories of a reduced five-level family (512
    parameter sets, 80 steps each, all generated in one persistent launch
    per step), roll out 16 held-out sets, judge every rollout by its TTNS
    run at trace distance 1e-3 and fall back to TTNS when rejected.

    Asserted: training lowers the loss 10x; the trained network's one-step
    prediction on held-out sets beats free propagation of the electronic
    system (the method without the bath) and the untrained network; every
    delivered trajectory is within the tolerance of TTNS (the fallback
    guarantee); a rollout takes less time than the TTNS run it would
    replace.  Printed: the accepted count and the multi-step errors."""
    import math
    import torch
    N = _N()
    steps, window, tol, n_train, n_test = 80, 8, 1e-3, 512, 16
    fam = dict(L=4, d=5, D=5, steps=steps)
    train = W.learned_sets(100000, n_train, **fam)
    test = W.learned_sets(200000, n_test, **fam)
    models = train + test
    rdm, t_ttns = _ttns_trajectories(models, steps)
    n = rdm.shape[-1]
    nc = N.conditioning(train[0]).size
    B = 1024
    cfg = N.config(n, window, nc, 128, 3, B, 1)
    sizes = OL.layer_sizes(window, n * n, nc, 128, 3, True)
    p0 = OL.flatten(OL.init_params(sizes, np.random.default_rng(7), True)).astype(np.float32)
    net = N.Net(cfg, p0)
    enc = net.ttnn_encode(torch.from_numpy(rdm).to("cuda"))  # (sets, steps + 1, n^2)
    cond = torch.from_numpy(np.stack([N.conditioning(m) for m in models])).to("cuda")
    props = torch.from_numpy(np.stack([N.propagator(m, m["dt"]) for m in models])).to("cuda")
    net.ttnn_set_data(enc[:n_train].contiguous(), cond[:n_train].contiguous(), props[:n_train].contiguous())
    rng = np.random.default_rng(8)

    def smp():
        return np.stack([rng.integers(0, n_train, B), rng.integers(window - 1, steps, B)], axis=1).astype(np.int32)

    loss0, _ = net.ttnn_gradients(smp())
    iters = 20000
    for it in range(iters):
        lr = 1e-6 + 0.5 * (1e-3 - 1e-6) * (1 + math.cos(math.pi * it / iters))
        net.ttnn_train_step(smp(), lr)
    loss1 = net.ttnn_last_loss()
    assert loss1 < 0.1 * loss0, (loss0, loss1)

    te = enc[n_train:]
    init = te[:, :window].contiguous()
    ref = te[:, window:].contiguous()
    cte, pte = cond[n_train:].contiguous(), props[n_train:].contiguous()
    n_roll = steps + 1 - window
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = net.ttnn_rollout(init, cte, n_roll, pte)
    torch.cuda.synchronize()
    t_roll = time.perf_counter() - t0
    dist, worst, accept = net.ttnn_judge(pred, ref, tol)
    final = net.ttnn_select(pred, ref, accept)
    # every delivered trajectory is within tol of TTNS (oracle trace distance)
    dfin = OL.trace_distance(OL.decode(final.cpu().numpy().astype(np.float64), n),
                             OL.decode(ref.cpu().numpy().astype(np.float64), n))
    assert dfin.max() <= tol + 1e-6
    d_tr = dist.cpu().numpy()
    # baselines: free propagation (zero network) and the untrained network
    net.ttnn_set_params(np.zeros_like(p0))
    d_free, _, _ = net.ttnn_judge(net.ttnn_rollout(init, cte, n_roll, pte), ref, tol)
    net.ttnn_set_params(p0)
    d_un, _, _ = net.ttnn_judge(net.ttnn_rollout(init, cte, n_roll, pte), ref, tol)
    d_free, d_un = d_free.cpu().numpy(), d_un.cpu().numpy()
    print("learned form: loss %.3e -> %.3e; held-out one-step trace distance trained %.2e, free propagation "
          "%.2e, untrained %.2e; after 10 steps %.2e / %.2e / %.2e; worst over %d steps %.2e / %.2e; "
          "accepted %d/%d at %.0e; rollout %.1f ms vs TTNS %.1f ms (%d sets in one batch)"
          % (loss0, loss1, np.median(d_tr[:, 0]), np.median(d_free[:, 0]), np.median(d_un[:, 0]),
             np.median(d_tr[:, 10]), np.median(d_free[:, 10]), np.median(d_un[:, 10]), n_roll,
             np.median(d_tr.max(1)), np.median(d_free.max(1)), int(accept.sum()), n_test, tol, 1e3 * t_roll,
             1e3 * t_ttns, len(models)))
    assert np.median(d_tr[:, 0]) < 0.7 * np.median(d_free[:, 0])
    assert np.median(d_tr[:, 0]) < 0.7 * np.median(d_un[:, 0])
    assert t_roll < t_ttns
    net.close()

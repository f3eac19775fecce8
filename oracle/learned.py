"""Learned propagator of the electronic reduced density matrix (CPU oracle,
test infrastructure).

A transfer-tensor-style map: the next reduced density matrix (RDM) of the
electronic root is predicted from the last M RDMs of the trajectory and the
parameters of the model, with a small multilayer perceptron.  The paper's
only learning component is the k-means clustering of its vibronic couplings
(section "Interface to TTNS"); this propagator is an addition whose training
data are RDM trajectories the TTNS-TDVP method itself generates, and whose
every prediction is judged against (and can fall back to) the full method.

Encoding of an n x n Hermitian RDM into n^2 reals: the n diagonal entries,
then Re rho_jk and then Im rho_jk for j < k in row-major order.

Network (plain FP64 here):
    x = [enc(rho_{t-M+1}) ... enc(rho_t), conditioning]
    h_1 = tanh(W_1 x + b_1), h_2 = tanh(W_2 h_1 + b_2), h_3 = tanh(W_3 h_2 + b_3)
    enc(rho_{t+1}) ~ enc(U rho_t U^dagger) + W_4 h_3 + b_4   (residual prediction)
where U = exp(-i H_S dt) is the free propagator of the electronic system
(the identity when no propagator is given): the network learns only what the
environment adds to the known system dynamics, as a transfer-tensor scheme
learns a memory kernel on top of the free evolution.

With the linear skip (``skip=True``) the input also carries the products
cond_c * enc(rho_t)_e (row-major over (c, e)), and the output adds a linear
map of the whole input, W_s x (no bias): a transfer-tensor-like linear term
whose coefficients depend on the model parameters, with the MLP on top.
Loss: mean squared error over the batch and the n^2 outputs.  Optimiser:
Adam (Kingma & Ba 2015) with bias correction.
Rollout: predict, decode, divide by the trace, shift the window.
Trace distance: half the sum of the absolute eigenvalues of rho - sigma.
"""
import numpy as np
import scipy.linalg

BETA1, BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


def encode(rho):
    """(..., n, n) Hermitian -> (..., n^2) reals."""
    rho = np.asarray(rho)
    n = rho.shape[-1]
    iu = np.triu_indices(n, 1)
    diag = np.real(np.diagonal(rho, axis1=-2, axis2=-1))
    up = rho[..., iu[0], iu[1]]
    return np.concatenate([diag, up.real, up.imag], axis=-1)


def decode(v, n):
    v = np.asarray(v, dtype=np.float64)
    m = n * (n - 1) // 2
    rho = np.zeros(v.shape[:-1] + (n, n), dtype=np.complex128)
    idx = np.arange(n)
    rho[..., idx, idx] = v[..., :n]
    iu = np.triu_indices(n, 1)
    up = v[..., n:n + m] + 1j * v[..., n + m:n + 2 * m]
    rho[..., iu[0], iu[1]] = up
    rho[..., iu[1], iu[0]] = np.conj(up)
    return rho


def propagator(model, dt):
    """U = exp(-i H_S dt) of the electronic system Hamiltonian."""
    return scipy.linalg.expm(-1j * np.asarray(model["h_el"], dtype=np.complex128) * dt)


def propagate(enc, U, n):
    """enc(U rho U^dagger) for encoded rho (..., n^2) and U (..., n, n)."""
    rho = decode(enc, n)
    return encode(U @ rho @ np.conj(np.swapaxes(U, -1, -2)))


def conditioning(model):
    """Model parameters as reals: H_S diagonal, H_S upper triangle (real
    part, row-major), alpha of each chain, diagonal of each coupling."""
    h = np.asarray(model["h_el"])
    n = h.shape[0]
    iu = np.triu_indices(n, 1)
    parts = [h.real[np.arange(n), np.arange(n)], h.real[iu]]
    parts.append(np.array([c["alpha"] for c in model["chains"]]))
    for c in model["chains"]:
        parts.append(np.real(np.diag(np.asarray(c["coupling"]))))
    return np.concatenate(parts).astype(np.float64)


def input_size(window, n_enc, n_cond, skip=False):
    return window * n_enc + n_cond + (n_cond * n_enc if skip else 0)


def layer_sizes(window, n_enc, n_cond, hidden, layers, skip=False):
    return [input_size(window, n_enc, n_cond, skip)] + [hidden] * layers + [n_enc]


def init_params(sizes, rng, skip=False):
    """Weights N(0, 1/fan_in), biases zero; list of (W, b), W of shape
    (fan_out, fan_in); with the skip a last (W_s, None), W_s zero
    (n_enc x input)."""
    p = [(rng.normal(0.0, 1.0 / np.sqrt(a), size=(b, a)), np.zeros(b))
         for a, b in zip(sizes[:-1], sizes[1:])]
    if skip:
        p.append((np.zeros((sizes[-1], sizes[0])), None))
    return p


def flatten(params):
    return np.concatenate([np.concatenate([W.reshape(-1)] + ([] if b is None else [b])) for W, b in params])


def unflatten(flat, sizes, skip=False):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + a * b].reshape(b, a)
        o += a * b
        bb = flat[o:o + b]
        o += b
        out.append((W, bb))
    if skip:
        out.append((flat[o:o + sizes[-1] * sizes[0]].reshape(sizes[-1], sizes[0]), None))
    return out


def _has_skip(params):
    return params[-1][1] is None


def bilinear(cond, last):
    """cond_c * enc_e for every (c, e), row-major: (B, n_cond * n_enc)."""
    return (np.asarray(cond)[:, :, None] * np.asarray(last)[:, None, :]).reshape(len(cond), -1)


def windows(traj_enc, cond, samples, window, props=None, n=None, skip=False):
    """Training pairs: traj_enc (S, T, n_enc), cond (S, n_cond), samples
    (B, 2) of (trajectory, t) with t >= window - 1 and t + 1 < T.
    Returns X (B, window*n_enc + n_cond), Y (B, n_enc) = enc(rho_{t+1}) and
    the residual base R (B, n_enc): enc(U_s rho_t U_s^dagger) with the
    propagators props (S, n, n), or enc(rho_t) without."""
    X, Y, R = [], [], []
    for s, t in samples:
        w = traj_enc[s, t - window + 1:t + 1].reshape(-1)
        extra = [bilinear(cond[s][None], traj_enc[s, t][None])[0]] if skip else []
        X.append(np.concatenate([w, cond[s]] + extra))
        Y.append(traj_enc[s, t + 1])
        R.append(traj_enc[s, t] if props is None else propagate(traj_enc[s, t], props[s], n))
    return np.array(X), np.array(Y), np.array(R)


def forward(params, X, n_enc, window, resid=None):
    """resid: residual base (B, n_enc); default the last RDM of the window."""
    skip = _has_skip(params)
    mlp = params[:-1] if skip else params
    acts = [X]
    h = X
    for W, b in mlp[:-1]:
        h = np.tanh(h @ W.T + b)
        acts.append(h)
    W, b = mlp[-1]
    base = X[:, (window - 1) * n_enc:window * n_enc] if resid is None else resid
    out = base + h @ W.T + b
    if skip:
        out = out + X @ params[-1][0].T
    return out, acts


def loss_and_grads(params, X, Y, n_enc, window, resid=None):
    pred, acts = forward(params, X, n_enc, window, resid)
    diff = pred - Y
    loss = float(np.mean(diff ** 2))
    g = 2.0 * diff / diff.size
    skip = _has_skip(params)
    mlp = params[:-1] if skip else params
    grads = [None] * len(params)
    if skip:
        grads[-1] = (g.T @ X, None)
    for li in range(len(mlp) - 1, -1, -1):
        W, b = mlp[li]
        a_in = acts[li]
        grads[li] = (g.T @ a_in, g.sum(axis=0))
        if li > 0:
            g = (g @ W) * (1.0 - a_in ** 2)
    return loss, grads


def adam_step(params, grads, m, v, t, lr):
    """One Adam update (t counts from 1); m, v lists like params."""
    new_p, new_m, new_v = [], [], []
    c1, c2 = 1.0 - BETA1 ** t, 1.0 - BETA2 ** t
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            if p is None:
                out.append((None, None, None))
                continue
            mm = BETA1 * mm + (1 - BETA1) * g
            vv = BETA2 * vv + (1 - BETA2) * g * g
            p = p - lr * (mm / c1) / (np.sqrt(vv / c2) + ADAM_EPS)
            out.append((p, mm, vv))
        new_p.append((out[0][0], out[1][0]))
        new_m.append((out[0][1], out[1][1]))
        new_v.append((out[0][2], out[1][2]))
    return new_p, new_m, new_v


def rollout(params, init_enc, cond, n_steps, n, window, props=None):
    """init_enc (B, window, n_enc): the last `window` RDMs; props (B, n, n)
    or None; returns (B, n_steps, n_enc): predicted, decoded,
    trace-renormalised RDMs."""
    w = np.array(init_enc, dtype=np.float64)
    cond = np.asarray(cond, dtype=np.float64)
    skip = _has_skip(params)
    out = []
    for _ in range(n_steps):
        parts = [w.reshape(w.shape[0], -1), cond] + ([bilinear(cond, w[:, -1])] if skip else [])
        X = np.concatenate(parts, axis=1)
        resid = None if props is None else propagate(w[:, -1], props, n)
        pred, _ = forward(params, X, n * n, window, resid)
        rho = decode(pred, n)
        tr = np.real(np.trace(rho, axis1=-2, axis2=-1))
        rho = rho / tr[:, None, None]
        e = encode(rho)
        out.append(e)
        w = np.concatenate([w[:, 1:], e[:, None, :]], axis=1)
    return np.stack(out, axis=1)


def trace_distance(rho, sigma):
    ev = np.linalg.eigvalsh(np.asarray(rho) - np.asarray(sigma))
    return 0.5 * np.sum(np.abs(ev), axis=-1)

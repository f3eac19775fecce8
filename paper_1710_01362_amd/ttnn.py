"""Thin ctypes binding of the learned RDM propagator (include/ttnn.h).

Argument marshalling only: training (forward, loss, backward, Adam),
rollouts, encoding and judging run in the HIP library.  PyTorch provides the
device workspace and the stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import ttns as T

EXPORTED = [
    "ttnn_param_count", "ttnn_workspace_size", "ttnn_build", "ttnn_conditioning", "ttnn_propagator",
    "ttnn_encode",
    "ttnn_set_data", "ttnn_gradients", "ttnn_train_step", "ttnn_last_loss", "ttnn_get_params",
    "ttnn_set_params", "ttnn_rollout", "ttnn_judge", "ttnn_select", "ttnn_destroy",
]


class Config(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("window", C.c_int32), ("n_cond", C.c_int32),
                ("hidden", C.c_int32), ("layers", C.c_int32), ("max_batch", C.c_int32),
                ("skip", C.c_int32)]


_ready = False


def lib():
    global _ready
    L = T.lib()
    if not _ready:
        P, I, S, F = C.c_void_p, C.c_int32, C.c_size_t, C.c_float
        L.ttnn_param_count.argtypes = [C.POINTER(Config), C.POINTER(C.c_int64)]
        L.ttnn_workspace_size.argtypes = [C.POINTER(Config), C.POINTER(S)]
        L.ttnn_build.argtypes = [C.POINTER(Config), P, P, S, P, C.POINTER(P)]
        L.ttnn_conditioning.argtypes = [C.POINTER(T.StarModel), P, I, C.POINTER(I)]
        L.ttnn_propagator.argtypes = [C.POINTER(T.StarModel), C.c_double, P, I]
        L.ttnn_encode.argtypes = [P, P, C.c_int64, P]
        L.ttnn_set_data.argtypes = [P, P, P, P, I, I]
        L.ttnn_gradients.argtypes = [P, P, I, P, P]
        L.ttnn_train_step.argtypes = [P, P, I, F, P]
        L.ttnn_last_loss.argtypes = [P, P]
        L.ttnn_get_params.argtypes = [P, P]
        L.ttnn_set_params.argtypes = [P, P]
        L.ttnn_rollout.argtypes = [P, P, P, P, I, I, P]
        L.ttnn_judge.argtypes = [P, P, P, I, I, F, P, P, P]
        L.ttnn_select.argtypes = [P, P, P, P, I, I, P]
        L.ttnn_destroy.argtypes = [P]
        for name in EXPORTED:
            getattr(L, name).restype = C.c_int
        _ready = True
    return L


def config(n_levels, window, n_cond, hidden, layers, max_batch, skip=0):
    return Config(n_levels, window, n_cond, hidden, layers, max_batch, int(skip))


def param_count(cfg):
    n = C.c_int64()
    T.check(lib().ttnn_param_count(C.byref(cfg), C.byref(n)))
    return n.value


def workspace_size(cfg):
    n = C.c_size_t()
    T.check(lib().ttnn_workspace_size(C.byref(cfg), C.byref(n)))
    return n.value


def conditioning(model):
    """Conditioning reals of a star model (workload dict), via the library."""
    keep = []
    sm = T.star_model(model, keep)
    out = np.zeros(4096, dtype=np.float32)
    n = C.c_int32()
    T.check(lib().ttnn_conditioning(C.byref(sm), out.ctypes.data, out.size, C.byref(n)))
    return out[:n.value].copy()


def propagator(model, dt):
    """Free propagator exp(-i H_S dt) of a star model (workload dict) as
    2 n^2 floats, via the library."""
    keep = []
    sm = T.star_model(model, keep)
    n = int(np.asarray(model["h_el"]).shape[0])
    out = np.zeros(2 * n * n, dtype=np.float32)
    T.check(lib().ttnn_propagator(C.byref(sm), C.c_double(dt), out.ctypes.data, out.size))
    return out


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _opt(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Net:
    """A network laid out in a PyTorch-owned device workspace."""

    def __init__(self, cfg, params, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.n_params = param_count(cfg)
        params = np.ascontiguousarray(params, dtype=np.float32)
        if params.size != self.n_params:
            raise ValueError("expected %d parameters, got %d" % (self.n_params, params.size))
        nbytes = workspace_size(cfg)
        self.device = torch.device(device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.net = C.c_void_p()
        T.check(lib().ttnn_build(C.byref(cfg), params.ctypes.data, C.c_void_p(base), C.c_size_t(nbytes),
                                 C.c_void_p(self.stream.cuda_stream), C.byref(self.net)))
        self._data = None

    def close(self):
        if self.net:
            lib().ttnn_destroy(self.net)
            self.net = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ttnn_encode(self, rdm_dev):
        """rdm_dev: complex128 device tensor (..., n, n) -> float32 (..., n^2)."""
        torch = self.torch
        n = self.cfg.n_levels
        src = torch.view_as_real(rdm_dev.contiguous()).contiguous()
        count = rdm_dev.numel() // (n * n)
        out = torch.empty(rdm_dev.shape[:-2] + (n * n,), dtype=torch.float32, device=self.device)
        T.check(lib().ttnn_encode(self.net, _ptr(src), count, _ptr(out)))
        return out

    def ttnn_set_data(self, traj_dev, cond_dev, prop_dev=None):
        """traj_dev: (sets, times, n^2) float32; cond_dev: (sets, n_cond)
        float32; prop_dev: (sets, 2 n^2) float32 free propagators or None."""
        self._data = (traj_dev.contiguous(), cond_dev.contiguous(),
                      None if prop_dev is None else prop_dev.contiguous())
        s, t = traj_dev.shape[0], traj_dev.shape[1]
        T.check(lib().ttnn_set_data(self.net, _ptr(self._data[0]), _ptr(self._data[1]), _opt(self._data[2]), s, t))

    def ttnn_gradients(self, samples):
        samples = np.ascontiguousarray(samples, dtype=np.int32)
        loss = np.zeros(1, dtype=np.float32)
        grad = np.zeros(self.n_params, dtype=np.float32)
        T.check(lib().ttnn_gradients(self.net, samples.ctypes.data, samples.shape[0], loss.ctypes.data,
                                     grad.ctypes.data))
        return float(loss[0]), grad

    def ttnn_train_step(self, samples, lr, noise_dev=None):
        """noise_dev: optional (B, window * n^2) float32 device tensor added to
        the input windows."""
        samples = np.ascontiguousarray(samples, dtype=np.int32)
        nz = None
        if noise_dev is not None:
            nz = noise_dev.contiguous()
            if nz.numel() != samples.shape[0] * self.cfg.window * self.cfg.n_levels ** 2:
                raise ValueError("noise must hold batch x window x n^2 floats")
            self._noise = nz
        T.check(lib().ttnn_train_step(self.net, samples.ctypes.data, samples.shape[0], C.c_float(lr),
                                      _ptr(nz) if nz is not None else None))

    def ttnn_last_loss(self):
        loss = np.zeros(1, dtype=np.float32)
        T.check(lib().ttnn_last_loss(self.net, loss.ctypes.data))
        return float(loss[0])

    def ttnn_get_params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        T.check(lib().ttnn_get_params(self.net, out.ctypes.data))
        return out

    def ttnn_set_params(self, params):
        params = np.ascontiguousarray(params, dtype=np.float32)
        T.check(lib().ttnn_set_params(self.net, params.ctypes.data))

    def ttnn_rollout(self, init_dev, cond_dev, n_steps, prop_dev=None):
        """init_dev: (B, window, n^2), cond_dev: (B, n_cond), prop_dev:
        (B, 2 n^2) or None -> (B, n_steps, n^2)."""
        torch = self.torch
        init_dev = init_dev.contiguous()
        cond_dev = cond_dev.contiguous()
        prop_dev = None if prop_dev is None else prop_dev.contiguous()
        B = init_dev.shape[0]
        out = torch.empty((B, n_steps, self.cfg.n_levels ** 2), dtype=torch.float32, device=self.device)
        T.check(lib().ttnn_rollout(self.net, _ptr(init_dev), _ptr(cond_dev), _opt(prop_dev), B, n_steps, _ptr(out)))
        return out

    def ttnn_judge(self, pred_dev, ref_dev, tol):
        torch = self.torch
        pred_dev = pred_dev.contiguous()
        ref_dev = ref_dev.contiguous()
        B, S = pred_dev.shape[0], pred_dev.shape[1]
        dist = torch.empty((B, S), dtype=torch.float32, device=self.device)
        worst = torch.empty(B, dtype=torch.float32, device=self.device)
        accept = torch.empty(B, dtype=torch.int32, device=self.device)
        T.check(lib().ttnn_judge(self.net, _ptr(pred_dev), _ptr(ref_dev), B, S, C.c_float(tol), _ptr(dist),
                                 _ptr(worst), _ptr(accept)))
        return dist, worst, accept

    def ttnn_select(self, pred_dev, ref_dev, accept_dev):
        torch = self.torch
        out = torch.empty_like(pred_dev)
        B, S = pred_dev.shape[0], pred_dev.shape[1]
        T.check(lib().ttnn_select(self.net, _ptr(pred_dev.contiguous()), _ptr(ref_dev.contiguous()),
                                  _ptr(accept_dev.contiguous()), B, S, _ptr(out)))
        return out

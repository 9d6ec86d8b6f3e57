"""Learned initialiser: binding of the network entry points of libvfisv.so
and the training loop that drives them.

The network, its kernels and the optimiser live in the library; this module
marshals device pointers and streams, draws the training set's random
parameters on the host (seeded numpy), and runs the epoch / early-stopping
loop of Sect. 5 (stop when the control-set error rises).
"""
import ctypes
import math
import os
import time

import numpy as np
import torch

from . import (NPAR, Context, Instrument, Options, VfisvError, _alloc_out, _Options, _out_ptrs,
               _ptr, _rows, _stream, _vp, _w_numel, lib, synthesize)

NCODE = 10


def _L():
    L = lib()
    if not getattr(L, "_mlp_sigs", False):
        fp = ctypes.POINTER(ctypes.c_float)
        L.vfisv_mlp_create.argtypes = [_vp, ctypes.c_int, fp, fp, fp, fp, ctypes.c_uint64,
                                       ctypes.POINTER(_vp)]
        L.vfisv_mlp_destroy.argtypes = [_vp]
        L.vfisv_mlp_num_params.argtypes = [_vp]
        L.vfisv_mlp_num_params.restype = ctypes.c_int64
        L.vfisv_mlp_num_inputs.argtypes = [_vp]
        L.vfisv_mlp_num_inputs.restype = ctypes.c_int
        L.vfisv_mlp_get_params.argtypes = [_vp, fp, ctypes.c_int64]
        L.vfisv_mlp_set_params.argtypes = [_vp, fp, ctypes.c_int64]
        L.vfisv_mlp_forward.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp]
        L.vfisv_mlp_gradient.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]
        L.vfisv_mlp_train_step.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_float,
                                           _vp]
        L.vfisv_mlp_take_loss.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
        L.vfisv_mlp_save.argtypes = [_vp, ctypes.c_char_p]
        L.vfisv_mlp_load.argtypes = [_vp, ctypes.c_char_p, ctypes.POINTER(_vp)]
        L.vfisv_invert_learned.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_int,
                                           ctypes.POINTER(_Options), ctypes.c_int,
                                           ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
        L._mlp_sigs = True
    return L


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Mlp:
    """A network in the library (weights on the context's device)."""

    def __init__(self, ctx, n_in=None, in_mean=None, in_std=None, out_mean=None, out_std=None,
                 seed=0, _handle=None):
        self.ctx = ctx
        if _handle is not None:
            self._h = _handle
            return
        keep = [_f32(x) for x in (in_mean, in_std, out_mean, out_std)]
        h = _vp()
        ctx._check(_L().vfisv_mlp_create(ctx._h, int(n_in), keep[0][1], keep[1][1], keep[2][1],
                                         keep[3][1], int(seed), ctypes.byref(h)),
                   "vfisv_mlp_create")
        self._h = h

    @classmethod
    def load(cls, ctx, path):
        h = _vp()
        ctx._check(_L().vfisv_mlp_load(ctx._h, os.fsencode(path), ctypes.byref(h)),
                   "vfisv_mlp_load")
        return cls(ctx, _handle=h)

    def save(self, path):
        self.ctx._check(_L().vfisv_mlp_save(self._h, os.fsencode(path)), "vfisv_mlp_save")

    def close(self):
        if getattr(self, "_h", None):
            _L().vfisv_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self):
        return int(_L().vfisv_mlp_num_params(self._h))

    @property
    def n_in(self):
        return int(_L().vfisv_mlp_num_inputs(self._h))

    def _input_rows(self, stokes):
        n = _rows(stokes)
        if stokes.numel() != n * self.n_in:
            raise ValueError("stokes must be [n, %d] for this network, got shape %s"
                             % (self.n_in, tuple(stokes.shape)))
        return n

    def get_params(self):
        a = np.empty(self.num_params, np.float32)
        self.ctx._check(_L().vfisv_mlp_get_params(
            self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size), "get_params")
        return a

    def set_params(self, a):
        a, p = _f32(a)
        self.ctx._check(_L().vfisv_mlp_set_params(self._h, p, a.size), "set_params")

    def forward(self, stokes, codes=True, params=True):
        dev = self.ctx.device
        n = self._input_rows(stokes)
        c = torch.empty((n, NCODE), device=dev, dtype=torch.float32) if codes else None
        p = torch.empty((n, NPAR), device=dev, dtype=torch.float32) if params else None
        self.ctx._check(_L().vfisv_mlp_forward(
            self.ctx._h, self._h, n, _ptr(stokes, torch.float32, dev, name="stokes"),
            _ptr(c, torch.float32, dev, name="codes"), _ptr(p, torch.float32, dev, name="params"),
            _stream(dev)), "vfisv_mlp_forward")
        return c, p

    def gradient(self, stokes, targets):
        dev = self.ctx.device
        n = self._input_rows(stokes)
        g = torch.empty(self.num_params, device=dev, dtype=torch.float32)
        loss = torch.empty(1, device=dev, dtype=torch.float64)
        self.ctx._check(_L().vfisv_mlp_gradient(
            self.ctx._h, self._h, n, _ptr(stokes, torch.float32, dev, name="stokes"),
            _ptr(targets, torch.float32, dev, n * NCODE, name="targets"),
            _ptr(g, torch.float32, dev),
            _ptr(loss, torch.float64, dev), _stream(dev)), "vfisv_mlp_gradient")
        return g, loss

    def train_step(self, stokes, targets, rows, lr, check_rows=True):
        """One Adam step on stokes[rows], targets[rows].  The library does not
        bound-check the indices; check_rows (one host synchronisation) does,
        for callers whose rows are not in range by construction."""
        dev = self.ctx.device
        n = self._input_rows(stokes)
        if rows.dim() != 1:
            raise ValueError("rows must be one-dimensional")
        if check_rows and rows.numel() and (int(rows.min()) < 0 or int(rows.max()) >= n):
            raise ValueError("rows must index the %d rows of stokes" % n)
        self.ctx._check(_L().vfisv_mlp_train_step(
            self.ctx._h, self._h, _ptr(stokes, torch.float32, dev, name="stokes"),
            _ptr(targets, torch.float32, dev, n * NCODE, name="targets"),
            _ptr(rows, torch.int32, dev, name="rows"), rows.shape[0], float(lr), _stream(dev)),
            "vfisv_mlp_train_step")

    def take_loss(self):
        s = ctypes.c_double()
        self.ctx._check(_L().vfisv_mlp_take_loss(self._h, ctypes.byref(s)), "take_loss")
        return s.value


def invert_learned(ctx, inst, mlp, stokes, W, opts=None, learned_max_iter=15, chi2_accept=0.0,
                   out=None):
    """Learned start + at most learned_max_iter LM trials, plain-LM fallback."""
    dev = ctx.device
    opts = opts or Options()
    n = _rows(stokes)
    if out is None:
        out = _alloc_out(n, dev)
    o = opts.c()
    ctx._check(_L().vfisv_invert_learned(
        ctx._h, inst._h, mlp._h, n,
        _ptr(stokes, torch.float32, dev, n * 4 * inst.n_obs, name="stokes"),
        _ptr(W, torch.float32, dev, _w_numel(W, n, inst.n_obs), name="W"),
        1 if W.dim() == 3 else 0, ctypes.byref(o), int(learned_max_iter), float(chi2_accept),
        *_out_ptrs(out, n, dev), _stream(dev)), "vfisv_invert_learned")
    return out


# ---- training ------------------------------------------------------------

def encode_targets(P):
    """Model parameters [n, 10] (numpy float64) -> the network's raw codes
    before output standardisation: field vector / 3000, then v .. alpha."""
    g = np.radians(P[:, 1])
    p2 = 2.0 * np.radians(P[:, 2])
    T = np.empty((P.shape[0], NCODE))
    T[:, 0] = P[:, 0] * np.cos(g) / 3000.0
    T[:, 1] = P[:, 0] * np.sin(g) * np.cos(p2) / 3000.0
    T[:, 2] = P[:, 0] * np.sin(g) * np.sin(p2) / 3000.0
    T[:, 3:] = P[:, 3:]
    return T


def make_training_set(ctx, inst, n, seed, draw_params, draw_noise, chunk=1 << 20):
    """Synthesise n noisy pixels on the device from parameters drawn on the
    host.  Returns (stokes [n, 4*n_obs] device, params [n, 10] numpy)."""
    dev = ctx.device
    n_obs = inst.n_obs
    stokes = torch.empty((n, 4 * n_obs), device=dev, dtype=torch.float32)
    P_all = np.empty((n, NPAR))
    for k, off in enumerate(range(0, n, chunk)):
        m = min(chunk, n - off)
        P = draw_params(m, (seed, k))
        P_all[off:off + m] = P
        noise = draw_noise(m, n_obs, (seed, k))
        synthesize(ctx, inst, torch.tensor(P.astype(np.float32), device=dev),
                   noise=torch.tensor(noise.astype(np.float32), device=dev),
                   out=stokes[off:off + m].view(m, 4, n_obs))
    return stokes, P_all


def train(ctx, inst, train_stokes, train_P, control_stokes, control_P, epochs=20, batch=4096,
          lr=1e-3, seed=0, log=print, min_lr_frac=0.02):
    """Adam with a cosine learning-rate schedule; the weights of the epoch
    with the lowest control-set error are kept (early stopping)."""
    dev = ctx.device
    n = train_stokes.shape[0]
    S = train_stokes.float()
    in_mean = S.mean(dim=0).cpu().numpy()
    in_std = S.std(dim=0).clamp_min(1e-6).cpu().numpy()
    raw = encode_targets(train_P)
    out_mean = raw[:, 3:].mean(axis=0)
    out_std = raw[:, 3:].std(axis=0)
    mlp = Mlp(ctx, train_stokes.shape[1], in_mean, in_std, out_mean, out_std, seed=seed)

    def std_codes(P):
        T = encode_targets(P)
        T[:, 3:] = (T[:, 3:] - out_mean) / out_std
        return torch.tensor(T.astype(np.float32), device=dev)

    T_train = std_codes(train_P)
    T_ctrl = std_codes(control_P)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    best = (math.inf, None, -1)
    history = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(torch.int32).to(dev)
        for b in range(steps_per_epoch):
            frac = step / max(total - 1, 1)
            cur = lr * (min_lr_frac + (1 - min_lr_frac) * 0.5 * (1 + math.cos(math.pi * frac)))
            # a permutation of range(n): in range by construction
            mlp.train_step(S, T_train, perm[b * batch:(b + 1) * batch], cur, check_rows=False)
            step += 1
        train_mse = mlp.take_loss() / (steps_per_epoch * batch * NCODE)
        c, _ = mlp.forward(control_stokes, codes=True, params=False)
        ctrl_mse = float(((c - T_ctrl) ** 2).mean())
        history.append((ep, train_mse, ctrl_mse, time.perf_counter() - t0))
        log("epoch %d  train mse %.5f  control mse %.5f  (%.1f s)" % history[-1])
        if ctrl_mse < best[0]:
            best = (ctrl_mse, mlp.get_params(), ep)
        elif ctrl_mse > best[0] * 1.02 and ep - best[2] >= 3:
            log("control error rising: stop")
            break
    mlp.set_params(best[1])
    return mlp, dict(history=history, best_epoch=best[2], best_control_mse=best[0],
                     seconds=time.perf_counter() - t0, steps=step)

"""Learned initialiser: binding of the network entry points of libvfisv.so.

The network, its kernels, the optimiser and the training run of Sect. 5
(epochs, shuffling, learning-rate schedule, early stopping on the control
set) live in the library; this module marshals device pointers and
streams, and draws the training set's random parameters on the host
(seeded numpy) for the library's synthesis.
"""
import ctypes
import os
import time

import numpy as np
import torch

from . import (NPAR, Context, Instrument, Options, VfisvError, _alloc_out, _Counters, _Options,
               _out_ptrs, _ptr, _rows, _stream, _vp, _w_numel, lib, synthesize)

NCODE = 10


class _TrainSpec(ctypes.Structure):
    _fields_ = [("stokes", _vp), ("params", _vp), ("n", ctypes.c_int64),
                ("ctrl_stokes", _vp), ("ctrl_params", _vp), ("n_ctrl", ctypes.c_int64),
                ("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_float),
                ("min_lr_frac", ctypes.c_float), ("seed", ctypes.c_uint64)]


class _LearnedPhases(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 5), ("short_fit", _Counters), ("refit", _Counters)]


class _TrainReport(ctypes.Structure):
    _fields_ = [("epochs_run", ctypes.c_int), ("best_epoch", ctypes.c_int),
                ("best_control_mse", ctypes.c_double), ("steps", ctypes.c_int64)]


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
        L.vfisv_mlp_get_norm.argtypes = [_vp, fp, fp, fp, fp]
        L.vfisv_mlp_load.argtypes = [_vp, ctypes.c_char_p, ctypes.POINTER(_vp)]
        fp_ = ctypes.POINTER(ctypes.c_float)
        dp_ = ctypes.POINTER(ctypes.c_double)
        L.vfisv_mlp_stats.argtypes = [_vp, ctypes.c_int64, ctypes.c_int, _vp, _vp, fp_, fp_, fp_,
                                      fp_, _vp]
        L.vfisv_mlp_train.argtypes = [_vp, _vp, ctypes.POINTER(_TrainSpec),
                                      ctypes.POINTER(_TrainReport), dp_, dp_, _vp]
        L.vfisv_invert_learned.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_int,
                                           ctypes.POINTER(_Options), ctypes.c_int,
                                           ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
        L.vfisv_invert_learned_noalloc.argtypes = L.vfisv_invert_learned.argtypes
        L.vfisv_learned_phase_timing.argtypes = [_vp, ctypes.c_int]
        L.vfisv_learned_phases_get.argtypes = [_vp, ctypes.POINTER(_LearnedPhases)]
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

    def get_norm(self):
        """(in_mean, in_std, out_mean, out_std) as float32 numpy arrays."""
        n = self.n_in
        arrs = [np.empty(n, np.float32), np.empty(n, np.float32), np.empty(7, np.float32),
                np.empty(7, np.float32)]
        ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) for a in arrs]
        self.ctx._check(_L().vfisv_mlp_get_norm(self._h, *ptrs), "vfisv_mlp_get_norm")
        return arrs

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


# largest batch of vfisv_invert_learned_noalloc (its fixed scratch)
NOALLOC_MAX_PIXELS = 524288


def invert_learned(ctx, inst, mlp, stokes, W, opts=None, learned_max_iter=15, chi2_accept=0.0,
                   out=None, noalloc=False):
    """Learned start + at most learned_max_iter LM trials, plain-LM fallback.
    noalloc: through vfisv_invert_learned_noalloc (fixed library scratch, no
    allocation; out must then be given by a caller that cannot allocate)."""
    dev = ctx.device
    opts = opts or Options()
    n = _rows(stokes)
    if out is None:
        out = _alloc_out(n, dev)
    o = opts.c()
    fn = _L().vfisv_invert_learned_noalloc if noalloc else _L().vfisv_invert_learned
    ctx._check(fn(
        ctx._h, inst._h, mlp._h, n,
        _ptr(stokes, torch.float32, dev, n * 4 * inst.n_obs, name="stokes"),
        _ptr(W, torch.float32, dev, _w_numel(W, n, inst.n_obs), name="W"),
        1 if W.dim() == 3 else 0, ctypes.byref(o), int(learned_max_iter), float(chi2_accept),
        *_out_ptrs(out, n, dev), _stream(dev)),
        "vfisv_invert_learned_noalloc" if noalloc else "vfisv_invert_learned")
    return out


PHASES = ("network", "short_fit", "select_combined", "refit", "merge")


def phase_timing(ctx, on=True):
    """Per-phase HIP-event timing of later learned-path calls (not captured
    ones): vfisv_learned_phase_timing."""
    ctx._check(_L().vfisv_learned_phase_timing(ctx._h, 1 if on else 0),
               "vfisv_learned_phase_timing")


def learned_phases(ctx):
    """The most recent timed learned-path call: {"ms": {phase: ms},
    "short_fit": counters, "refit": counters}."""
    r = _LearnedPhases()
    ctx._check(_L().vfisv_learned_phases_get(ctx._h, ctypes.byref(r)), "vfisv_learned_phases_get")

    def cnt(c):
        return {f: int(getattr(c, f)) for f, _ in _Counters._fields_}
    return {"ms": dict(zip(PHASES, list(r.ms))), "short_fit": cnt(r.short_fit),
            "refit": cnt(r.refit)}


# ---- training ------------------------------------------------------------

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


def _dev_params(P, dev):
    if isinstance(P, torch.Tensor):
        return P.to(device=dev, dtype=torch.float32).contiguous()
    return torch.tensor(np.ascontiguousarray(P, dtype=np.float32), device=dev)


def training_stats(ctx, stokes, P):
    """Normalisation of a training set (vfisv_mlp_stats): (in_mean, in_std)
    per input column and (out_mean, out_std) of v .. alpha, float32 numpy."""
    dev = ctx.device
    n = _rows(stokes)
    n_in = stokes.shape[1]
    Pd = _dev_params(P, dev)
    stats = [np.empty(n_in, np.float32), np.empty(n_in, np.float32), np.empty(7, np.float32),
             np.empty(7, np.float32)]
    fptr = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) for a in stats]
    ctx._check(_L().vfisv_mlp_stats(
        ctx._h, n, n_in, _ptr(stokes, torch.float32, dev, n * n_in, name="stokes"),
        _ptr(Pd, torch.float32, dev, n * NPAR, name="P"), *fptr, _stream(dev)),
        "vfisv_mlp_stats")
    return stats


def train_network(ctx, mlp, train_stokes, train_P, control_stokes, control_P, epochs=20,
                  batch=4096, lr=1e-3, seed=0, min_lr_frac=0.02):
    """vfisv_mlp_train on an existing network: returns the report as a dict
    with the per-epoch history [(epoch, train mse, control mse)]."""
    dev = ctx.device
    n, nc = _rows(train_stokes), _rows(control_stokes, "control_stokes")
    n_in = mlp.n_in
    Pt, Pc = _dev_params(train_P, dev), _dev_params(control_P, dev)
    spec = _TrainSpec(_ptr(train_stokes, torch.float32, dev, n * n_in, name="train_stokes"),
                      _ptr(Pt, torch.float32, dev, n * NPAR, name="train_P"), n,
                      _ptr(control_stokes, torch.float32, dev, nc * n_in, name="control_stokes"),
                      _ptr(Pc, torch.float32, dev, nc * NPAR, name="control_P"), nc,
                      int(epochs), int(batch), float(lr), float(min_lr_frac), int(seed))
    rep = _TrainReport()
    tr = np.zeros(epochs)
    ce = np.zeros(epochs)
    dptr = ctypes.POINTER(ctypes.c_double)
    t0 = time.perf_counter()
    ctx._check(_L().vfisv_mlp_train(ctx._h, mlp._h, ctypes.byref(spec), ctypes.byref(rep),
                                    tr.ctypes.data_as(dptr), ce.ctypes.data_as(dptr),
                                    _stream(dev)), "vfisv_mlp_train")
    return dict(history=[(e, float(tr[e]), float(ce[e])) for e in range(rep.epochs_run)],
                best_epoch=rep.best_epoch, best_control_mse=rep.best_control_mse,
                seconds=time.perf_counter() - t0, steps=rep.steps)


def train(ctx, inst, train_stokes, train_P, control_stokes, control_P, epochs=20, batch=4096,
          lr=1e-3, seed=0, log=print, min_lr_frac=0.02):
    """The library's training run on a new network: normalisation from the
    training set, then Adam with a cosine learning rate and early stopping
    on the control set, keeping the best epoch's weights.  train_P /
    control_P: the models [n, 10] (numpy or tensor)."""
    stats = training_stats(ctx, train_stokes, train_P)
    mlp = Mlp(ctx, train_stokes.shape[1], *stats, seed=seed)
    info = train_network(ctx, mlp, train_stokes, train_P, control_stokes, control_P,
                         epochs=epochs, batch=batch, lr=lr, seed=seed, min_lr_frac=min_lr_frac)
    for h in info["history"]:
        log("epoch %d  train mse %.5f  control mse %.5f" % h)
    info["stats"] = stats
    return mlp, info

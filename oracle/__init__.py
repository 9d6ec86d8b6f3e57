"""FP64 CPU oracle of the Milne-Eddington Stokes inversion -- TEST INFRASTRUCTURE.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It wraps ``liboracle.so`` (plain C, FP64; see
``oracle.h``) with ctypes and shares nothing with the GPU library.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
NPAR = 10
CONVERGED, MAX_ITER, STALLED, NONFINITE = 0, 1, 2, 3

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int32)


class _Instrument(ctypes.Structure):
    _fields_ = [("lambda0_A", ctypes.c_double), ("geff", ctypes.c_double),
                ("n_fine", ctypes.c_int), ("fine_offset_mA", _dp),
                ("n_obs", ctypes.c_int), ("filter", _dp), ("voigt", ctypes.c_int)]


class _Options(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("eps0", ctypes.c_double),
                ("eps_max", ctypes.c_double), ("rel_tol", ctypes.c_double),
                ("free_mask", ctypes.c_uint32), ("fixed_iters", ctypes.c_int),
                ("restarts", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("hess_reuse", ctypes.c_double)]


class _Counters(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_int64), ("derivs", ctypes.c_int64),
                ("solves", ctypes.c_int64), ("svd_fallbacks", ctypes.c_int64),
                ("hessians", ctypes.c_int64)]


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _LIB = bind(_build.LIB)
    return _LIB


def bind(path):
    """Load an oracle library and declare its C signatures."""
    L = ctypes.CDLL(path)
    L.orc_faddeeva_batch.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp]
    L.orc_zeeman_constant.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_zeeman_constant.restype = ctypes.c_double
    L.orc_synth_fine.argtypes = [ctypes.POINTER(_Instrument), _dp, _dp, _dp]
    L.orc_voigt_taylor_batch.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, _dp, _dp, _dp]
    L.orc_voigt_taylor_batch.restype = None
    L.orc_voigt_table_node.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
    L.orc_voigt_table_node.restype = None
    L.orc_forward.argtypes = [ctypes.POINTER(_Instrument), _dp, _dp, _dp]
    L.orc_project.argtypes = [_dp]
    L.orc_eps_decrease.argtypes = [ctypes.c_double]
    L.orc_eps_decrease.restype = ctypes.c_double
    L.orc_eps_increase.argtypes = [ctypes.c_double]
    L.orc_eps_increase.restype = ctypes.c_double
    L.orc_solve.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_uint32, _dp]
    L.orc_solve.restype = ctypes.c_int
    L.orc_default_init.argtypes = [_dp]
    L.orc_lm_pixel.argtypes = [ctypes.POINTER(_Instrument), ctypes.POINTER(_Options),
                               _fp, _fp, _dp, ctypes.c_int64, _dp, _dp, _ip, _ip,
                               ctypes.POINTER(_Counters)]
    L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    L.orc_splitmix64.restype = ctypes.c_uint64
    L.orc_restart_uniform.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                      ctypes.c_int]
    L.orc_restart_uniform.restype = ctypes.c_double
    L.orc_invert.argtypes = [ctypes.POINTER(_Instrument), ctypes.POINTER(_Options),
                             ctypes.c_int64, _fp, _fp, ctypes.c_int, _dp, _dp, _dp,
                             _ip, _ip, ctypes.POINTER(_Counters), ctypes.c_int]
    L.orc_invert.restype = ctypes.c_int
    L.orc_forward_batch.argtypes = [ctypes.POINTER(_Instrument), ctypes.c_int64, _dp,
                                    _dp, ctypes.c_int]
    L.orc_forward_batch.restype = ctypes.c_int
    return L


def _d(a):
    return a.ctypes.data_as(_dp)


def _f(a):
    return a.ctypes.data_as(_fp)


def _i(a):
    return a.ctypes.data_as(_ip)


class Instrument:
    """A line observed through a linear filter.

    lambda0_A, geff: line centre [A] and effective Lande factor.
    fine_offset_mA: [n_fine] synthesis grid (offsets from line centre, mA).
    filt: [n_obs, n_fine] filter matrix.
    """

    def __init__(self, lambda0_A, geff, fine_offset_mA, filt, voigt=0):
        self.fine = np.ascontiguousarray(fine_offset_mA, dtype=np.float64)
        self.filt = np.ascontiguousarray(filt, dtype=np.float64)
        assert self.filt.shape[1] == self.fine.shape[0]
        assert voigt in (0, 1, 2)
        self.lambda0_A = float(lambda0_A)
        self.geff = float(geff)
        self.n_fine = self.fine.shape[0]
        self.n_obs = self.filt.shape[0]
        self.voigt = voigt
        self.c = _Instrument(float(lambda0_A), float(geff), self.n_fine, _d(self.fine),
                             self.n_obs, _d(self.filt), int(voigt))


@dataclass
class Options:
    max_iter: int = 50
    eps0: float = 1e-3
    eps_max: float = 1e8
    rel_tol: float = 1e-5
    free_mask: int = 0x3FF
    fixed_iters: int = 0
    restarts: int = 0
    seed: int = 0
    hess_reuse: float = 0.0

    def c(self):
        return _Options(self.max_iter, self.eps0, self.eps_max, self.rel_tol, self.free_mask,
                        self.fixed_iters, self.restarts, self.seed, self.hess_reuse)


def faddeeva(u, a):
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    a = np.ascontiguousarray(np.broadcast_to(a, u.shape), dtype=np.float64)
    H = np.empty_like(u)
    F = np.empty_like(u)
    lib().orc_faddeeva_batch(u.size, _d(u), _d(a), _d(H), _d(F))
    return H, F


def voigt_taylor(order, u, a):
    """H, F from the Taylor table (Sect. 3.2, Eqs. 10-13) at order 1 or 2."""
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    a = np.ascontiguousarray(np.broadcast_to(a, u.shape), dtype=np.float64)
    H = np.empty_like(u)
    F = np.empty_like(u)
    lib().orc_voigt_taylor_batch(int(order), u.size, _d(u), _d(a), _d(H), _d(F))
    return H, F


def splitmix64(seed, c):
    """Output number c (from 0) of the SplitMix64 stream seeded with seed."""
    return int(lib().orc_splitmix64(seed, c))


def restart_uniform(seed, pixel, k, p):
    return float(lib().orc_restart_uniform(seed, pixel, k, p))


def voigt_table_node(i, j):
    h, f = ctypes.c_double(), ctypes.c_double()
    lib().orc_voigt_table_node(i, j, ctypes.byref(h), ctypes.byref(f))
    return h.value, f.value


def zeeman_constant(lambda0_A, geff):
    return lib().orc_zeeman_constant(lambda0_A, geff)


def synth_fine(inst, M, deriv=True):
    M = np.ascontiguousarray(M, dtype=np.float64)
    S = np.empty((4, inst.n_fine))
    dS = np.empty((4, inst.n_fine, NPAR)) if deriv else None
    lib().orc_synth_fine(ctypes.byref(inst.c), _d(M), _d(S), _d(dS) if deriv else None)
    return (S, dS) if deriv else S


def forward(inst, M, jac=False):
    M = np.ascontiguousarray(M, dtype=np.float64)
    S = np.empty((4, inst.n_obs))
    J = np.empty((4, inst.n_obs, NPAR)) if jac else None
    lib().orc_forward(ctypes.byref(inst.c), _d(M), _d(S), _d(J) if jac else None)
    return (S, J) if jac else S


def forward_batch(inst, params, nthreads=0):
    P = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, NPAR)
    out = np.empty((P.shape[0], 4, inst.n_obs))
    lib().orc_forward_batch(ctypes.byref(inst.c), P.shape[0], _d(P), _d(out), nthreads)
    return out


def project(M):
    M = np.array(M, dtype=np.float64)
    lib().orc_project(_d(M))
    return M


def eps_decrease(e):
    return lib().orc_eps_decrease(e)


def eps_increase(e):
    return lib().orc_eps_increase(e)


def solve(H, g, eps, free_mask=0x3FF):
    H = np.ascontiguousarray(H, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    d = np.empty(NPAR)
    code = lib().orc_solve(_d(H), _d(g), eps, free_mask, _d(d))
    return d, code


def default_init():
    M = np.empty(NPAR)
    lib().orc_default_init(_d(M))
    return M


def lm_pixel(inst, obs, W, M0=None, opts=None, pixel=0):
    opts = opts or Options()
    obs = np.ascontiguousarray(obs, dtype=np.float32)
    W = np.ascontiguousarray(W, dtype=np.float32)
    M0c = None if M0 is None else np.ascontiguousarray(M0, dtype=np.float64)
    M = np.empty(NPAR)
    chi2 = np.empty(1)
    it = np.empty(1, np.int32)
    st = np.empty(1, np.int32)
    cnt = _Counters()
    o = opts.c()
    lib().orc_lm_pixel(ctypes.byref(inst.c), ctypes.byref(o), _f(obs), _f(W),
                       _d(M0c) if M0c is not None else None, int(pixel), _d(M), _d(chi2),
                       _i(it),
                       _i(st), ctypes.byref(cnt))
    return dict(params=M, chi2=float(chi2[0]), iters=int(it[0]), status=int(st[0]),
                counters=dict(trials=cnt.trials, derivs=cnt.derivs, solves=cnt.solves,
                              svd_fallbacks=cnt.svd_fallbacks, hessians=cnt.hessians))


def invert(inst, stokes, W, init=None, opts=None, nthreads=0):
    """Invert n pixels.  stokes: [n, 4, n_obs] float32; W: [4, n_obs] or
    [n, 4, n_obs]; init: [n, 10] or None (default model)."""
    opts = opts or Options()
    stokes = np.ascontiguousarray(stokes, dtype=np.float32)
    n = stokes.shape[0]
    W = np.ascontiguousarray(W, dtype=np.float32)
    per_pixel = 1 if W.ndim == 3 else 0
    initc = None if init is None else np.ascontiguousarray(init, dtype=np.float64)
    params = np.empty((n, NPAR))
    chi2 = np.empty(n)
    iters = np.empty(n, np.int32)
    status = np.empty(n, np.int32)
    cnt = _Counters()
    o = opts.c()
    used = lib().orc_invert(ctypes.byref(inst.c), ctypes.byref(o), n, _f(stokes), _f(W),
                            per_pixel, _d(initc) if initc is not None else None,
                            _d(params), _d(chi2), _i(iters), _i(status), ctypes.byref(cnt),
                            nthreads)
    return dict(params=params, chi2=chi2, iters=iters, status=status, threads=used,
                counters=dict(trials=cnt.trials, derivs=cnt.derivs, solves=cnt.solves,
                              svd_fallbacks=cnt.svd_fallbacks, hessians=cnt.hessians))

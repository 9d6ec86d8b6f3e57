"""MI355X-native Milne-Eddington Stokes inverter (VFISV hot path).

Thin ctypes binding of ``libvfisv.so`` (C ABI in ``include/vfisv.h``).  Torch
is used only for device memory and streams: every step of the inversion runs
in the library's HIP kernels.  There is no CPU fallback: if the library or a
HIP device is missing, calls raise.
"""
import ctypes
import os
from dataclasses import dataclass

import torch  # loaded first so the library binds to the process's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvfisv.so")
NPAR = 10
CONVERGED, MAX_ITER, STALLED, NONFINITE = 0, 1, 2, 3
FALLBACK_USED = 16
# Options.fallback_rule bits (learned path)
REFIT_UNCONVERGED, REFIT_FROM_DEFAULT, REFIT_KEEP_REFIT = 1, 2, 4
PARAM_NAMES = ("B", "gamma", "psi", "v_los", "doppler_width", "damping", "eta0", "S0", "S1",
               "alpha")

_vp = ctypes.c_void_p


class VfisvError(RuntimeError):
    pass


class _InstDesc(ctypes.Structure):
    _fields_ = [("lambda0_A", ctypes.c_double), ("geff", ctypes.c_double),
                ("n_fine", ctypes.c_int), ("fine_offset_mA", ctypes.POINTER(ctypes.c_double)),
                ("n_obs", ctypes.c_int), ("filter", ctypes.POINTER(ctypes.c_double)),
                ("tap_threshold", ctypes.c_double)]


class _InstInfo(ctypes.Structure):
    _fields_ = [("n_active_fine", ctypes.c_int), ("n_taps", ctypes.c_int),
                ("max_dropped_rel", ctypes.c_double),
                ("cz_mA_per_G", ctypes.c_double), ("lm_register_rows", ctypes.c_int)]


class _Options(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("eps0", ctypes.c_double),
                ("eps_max", ctypes.c_double), ("rel_tol", ctypes.c_double),
                ("free_mask", ctypes.c_uint32), ("grid_waves", ctypes.c_int),
                ("chunk_log2", ctypes.c_int), ("lanes_per_pixel", ctypes.c_int),
                ("voigt", ctypes.c_int), ("fixed_iters", ctypes.c_int),
                ("restarts", ctypes.c_int), ("restart_seed", ctypes.c_uint64),
                ("hess_reuse", ctypes.c_double), ("fallback_rule", ctypes.c_uint32),
                ("deriv_split", ctypes.c_int)]


class _Batch(ctypes.Structure):
    _fields_ = [("inst", ctypes.c_void_p), ("n", ctypes.c_int64), ("stokes", ctypes.c_void_p),
                ("W", ctypes.c_void_p), ("W_per_pixel", ctypes.c_int),
                ("init", ctypes.c_void_p), ("params", ctypes.c_void_p),
                ("chi2", ctypes.c_void_p), ("iters", ctypes.c_void_p),
                ("status", ctypes.c_void_p)]


class _Tuning(ctypes.Structure):
    _fields_ = [("grid_waves", ctypes.c_int), ("chunk_log2", ctypes.c_int),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("candidates", ctypes.c_int), ("sample", ctypes.c_int64),
                ("deriv_split", ctypes.c_int)]


class _Counters(ctypes.Structure):
    _fields_ = [("pixels", ctypes.c_int64), ("trials", ctypes.c_int64),
                ("accepts", ctypes.c_int64), ("passes", ctypes.c_int64),
                ("svd_fallbacks", ctypes.c_int64), ("grid_waves", ctypes.c_int64),
                ("hessians", ctypes.c_int64), ("derivative_passes", ctypes.c_int64),
                ("jacobians", ctypes.c_int64)]


# Every symbol declared in include/vfisv.h.
EXPORTS = ("vfisv_create", "vfisv_destroy", "vfisv_last_error", "vfisv_version",
           "vfisv_instrument_create", "vfisv_instrument_info_get", "vfisv_instrument_destroy",
           "vfisv_options_default", "vfisv_synthesize", "vfisv_invert", "vfisv_get_counters",
           "vfisv_solve", "vfisv_mlp_create", "vfisv_mlp_destroy", "vfisv_mlp_num_params", "vfisv_mlp_num_inputs", "vfisv_mlp_stats", "vfisv_mlp_train",
           "vfisv_mlp_get_params", "vfisv_mlp_set_params", "vfisv_mlp_forward",
           "vfisv_mlp_gradient", "vfisv_mlp_train_step", "vfisv_mlp_take_loss", "vfisv_mlp_save",
           "vfisv_mlp_load", "vfisv_invert_learned", "vfisv_invert_learned_noalloc",
           "vfisv_chi2_quantile", "vfisv_mlp_get_norm", "vfisv_learned_phase_timing", "vfisv_learned_phases_get",
           "vfisv_iter_histogram",
           "vfisv_invert_batches", "vfisv_autotune", "vfisv_synthesize_voigt",
           "vfisv_init_classical", "vfisv_init_combined", "vfisv_stokes_weights")

_LIB = None


def lib():
    """Load libvfisv.so (built by ``__graft_entry__.build()``)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise VfisvError("libvfisv.so is not built (%s); run __graft_entry__.build()"
                             % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.vfisv_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
        L.vfisv_destroy.argtypes = [_vp]
        L.vfisv_last_error.argtypes = [_vp]
        L.vfisv_last_error.restype = ctypes.c_char_p
        L.vfisv_version.restype = ctypes.c_char_p
        L.vfisv_instrument_create.argtypes = [_vp, ctypes.POINTER(_InstDesc), ctypes.POINTER(_vp)]
        L.vfisv_instrument_info_get.argtypes = [_vp, ctypes.POINTER(_InstInfo)]
        L.vfisv_instrument_destroy.argtypes = [_vp]
        L.vfisv_options_default.argtypes = [ctypes.POINTER(_Options)]
        L.vfisv_options_default.restype = None
        L.vfisv_synthesize.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]
        L.vfisv_synthesize_voigt.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp,
                                             ctypes.c_int, _vp]
        L.vfisv_invert.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_int, _vp,
                                   ctypes.POINTER(_Options), _vp, _vp, _vp, _vp, _vp]
        L.vfisv_get_counters.argtypes = [_vp, ctypes.POINTER(_Counters)]
        L.vfisv_solve.argtypes = [_vp, ctypes.c_int64, _vp, _vp, _vp, ctypes.c_uint32, _vp,
                                  _vp, _vp]
        L.vfisv_iter_histogram.argtypes = [_vp, ctypes.c_int64, _vp, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int64), _vp]
        L.vfisv_invert_batches.argtypes = [_vp, ctypes.POINTER(_Batch), ctypes.c_int,
                                           ctypes.POINTER(_Options), _vp]
        L.vfisv_init_classical.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp]
        L.vfisv_stokes_weights.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp,
                                           ctypes.POINTER(ctypes.c_float), _vp, _vp]
        L.vfisv_init_combined.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_float,
                                          _vp, _vp, _vp]
        L.vfisv_autotune.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_int,
                                     ctypes.POINTER(_Options), ctypes.c_int64,
                                     ctypes.POINTER(_Tuning), _vp]
        _LIB = L
    return _LIB


def version():
    return lib().vfisv_version().decode()


def _ptr(t, dtype, device, numel=None, name="tensor"):
    """Device address of a contiguous tensor, after checking its dtype,
    device and (when given) element count: the library takes bare pointers
    and reads or writes exactly the sizes its arguments imply."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.device != device:
        raise ValueError("%s must live on %s, got %s" % (name, device, t.device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must hold %d elements, got shape %s" % (name, numel, tuple(t.shape)))
    return t.data_ptr()


def _rows(t, name="stokes"):
    if not isinstance(t, torch.Tensor) or t.dim() < 1:
        raise TypeError("%s must be a torch tensor with a leading pixel dimension" % name)
    return t.shape[0]


def _w_numel(W, n, n_obs):
    return (n if W.dim() == 3 else 1) * 4 * n_obs


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


class Context:
    """Library context on one HIP device."""

    def __init__(self, device=0):
        if not torch.cuda.is_available():
            raise VfisvError("no HIP device visible")
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        h = _vp()
        rc = lib().vfisv_create(ctypes.byref(h), device)
        if rc != 0:
            raise VfisvError("vfisv_create: %s" % lib().vfisv_last_error(None).decode())
        self._h = h

    def _check(self, rc, what):
        if rc != 0:
            raise VfisvError("%s (rc %d): %s" % (what, rc,
                                                   lib().vfisv_last_error(self._h).decode()))

    def close(self):
        if getattr(self, "_h", None):
            lib().vfisv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def counters(self):
        c = _Counters()
        self._check(lib().vfisv_get_counters(self._h, ctypes.byref(c)), "vfisv_get_counters")
        return {k: getattr(c, k) for k, _ in _Counters._fields_}


class Instrument:
    """Line + synthesis grid + filter, copied to the device."""

    def __init__(self, ctx, lambda0_A, geff, fine_offset_mA, filt, tap_threshold=2.0 ** -24):
        import numpy as np
        self.ctx = ctx
        self._fine = np.ascontiguousarray(fine_offset_mA, dtype=np.float64)
        self._filt = np.ascontiguousarray(filt, dtype=np.float64)
        self.n_fine = int(self._fine.shape[0])
        self.n_obs = int(self._filt.shape[0])
        if self._filt.shape != (self.n_obs, self.n_fine):
            raise ValueError("filter must be [n_obs, n_fine]")
        d = _InstDesc(float(lambda0_A), float(geff), self.n_fine,
                      self._fine.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.n_obs,
                      self._filt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      float(tap_threshold))
        h = _vp()
        ctx._check(lib().vfisv_instrument_create(ctx._h, ctypes.byref(d), ctypes.byref(h)),
                   "vfisv_instrument_create")
        self._h = h
        info = _InstInfo()
        lib().vfisv_instrument_info_get(h, ctypes.byref(info))
        self.info = {k: getattr(info, k) for k, _ in _InstInfo._fields_}

    @classmethod
    def from_spec(cls, ctx, spec, **kw):
        return cls(ctx, spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().vfisv_instrument_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Options:
    max_iter: int = 50
    eps0: float = 1e-3
    eps_max: float = 1e8
    rel_tol: float = 1e-5
    free_mask: int = 0x3FF
    grid_waves: int = 0
    chunk_log2: int = -1
    lanes_per_pixel: int = 1
    voigt: int = 0
    fixed_iters: int = 0
    restarts: int = 0
    restart_seed: int = 0
    hess_reuse: float = 0.0
    fallback_rule: int = 0
    deriv_split: int = -1

    def c(self):
        return _Options(self.max_iter, self.eps0, self.eps_max, self.rel_tol, self.free_mask,
                        self.grid_waves, self.chunk_log2, self.lanes_per_pixel, self.voigt,
                        self.fixed_iters, self.restarts, self.restart_seed, self.hess_reuse,
                        self.fallback_rule, self.deriv_split)


def synthesize(ctx, inst, params, noise=None, jac=False, out=None, voigt=0):
    """Filtered Stokes vector [n, 4, n_obs] (and Jacobian [n, 4, n_obs, 10])
    of the models ``params`` [n, 10] (float32, on the context's device);
    ``voigt`` selects the H/F evaluation as Options.voigt does."""
    dev = ctx.device
    n = _rows(params, "params")
    m = n * 4 * inst.n_obs
    p = _ptr(params, torch.float32, dev, n * NPAR, name="params")
    stokes = out if out is not None else torch.empty((n, 4, inst.n_obs), device=dev,
                                                     dtype=torch.float32)
    J = torch.empty((n, 4, inst.n_obs, NPAR), device=dev, dtype=torch.float32) if jac else None
    ctx._check(lib().vfisv_synthesize_voigt(ctx._h, inst._h, n, p,
                                            _ptr(noise, torch.float32, dev, m, name="noise"),
                                            _ptr(stokes, torch.float32, dev, m, name="out"),
                                            _ptr(J, torch.float32, dev, m * NPAR, name="jac"),
                                            int(voigt),
                                            _stream(dev)),
               "vfisv_synthesize_voigt")
    return (stokes, J) if jac else stokes


def invert(ctx, inst, stokes, W, init=None, opts=None, out=None):
    """Invert n pixels: stokes [n, 4, n_obs] float32; W [4, n_obs] or
    [n, 4, n_obs] float32; init [n, 10] float32 or None.  Returns a dict of
    device tensors params [n, 10], chi2 [n] (float64), iters [n], status [n]."""
    dev = ctx.device
    opts = opts or Options()
    n = _rows(stokes)
    if out is None:
        out = _alloc_out(n, dev)
    per_pixel = 1 if W.dim() == 3 else 0
    o = opts.c()
    ctx._check(lib().vfisv_invert(
        ctx._h, inst._h, n, _ptr(stokes, torch.float32, dev, n * 4 * inst.n_obs, name="stokes"),
        _ptr(W, torch.float32, dev, _w_numel(W, n, inst.n_obs), name="W"), per_pixel,
        _ptr(init, torch.float32, dev, n * NPAR, name="init"), ctypes.byref(o),
        *_out_ptrs(out, n, dev), _stream(dev)), "vfisv_invert")
    return out


def _alloc_out(n, dev):
    return dict(params=torch.empty((n, NPAR), device=dev, dtype=torch.float32),
                chi2=torch.empty(n, device=dev, dtype=torch.float64),
                iters=torch.empty(n, device=dev, dtype=torch.int32),
                status=torch.empty(n, device=dev, dtype=torch.int32))


def _out_ptrs(out, n, dev):
    return (_ptr(out["params"], torch.float32, dev, n * NPAR, name="params"),
            _ptr(out["chi2"], torch.float64, dev, n, name="chi2"),
            _ptr(out["iters"], torch.int32, dev, n, name="iters"),
            _ptr(out["status"], torch.int32, dev, n, name="status"))


def invert_batches(ctx, batches, opts=None):
    """Several batches in one launch.  ``batches``: list of dicts with keys
    inst, stokes [n, 4, n_obs], W ([4, n_obs] or [n, 4, n_obs]), and
    optionally init [n, 10] and out (as returned by ``invert``).  Returns
    the list of output dicts, in order."""
    dev = ctx.device
    opts = opts or Options()
    arr = (_Batch * len(batches))()
    outs = []
    for i, b in enumerate(batches):
        n = _rows(b["stokes"])
        out = b.get("out") or _alloc_out(n, dev)
        outs.append(out)
        W = b["W"]
        inst = b["inst"]
        h = inst._h
        arr[i] = _Batch(h.value if isinstance(h, ctypes.c_void_p) else h, n,
                        _ptr(b["stokes"], torch.float32, dev, n * 4 * inst.n_obs, name="stokes"),
                        _ptr(W, torch.float32, dev, _w_numel(W, n, inst.n_obs), name="W"),
                        1 if W.dim() == 3 else 0,
                        _ptr(b.get("init"), torch.float32, dev, n * NPAR, name="init"),
                        *_out_ptrs(out, n, dev))
    o = opts.c()
    ctx._check(lib().vfisv_invert_batches(ctx._h, arr, len(batches), ctypes.byref(o),
                                          _stream(dev)), "vfisv_invert_batches")
    return outs


def init_classical(ctx, inst, stokes):
    """Classical starting models [n, 10] (weak field, azimuth, line
    position) and polarisation levels [n] for stokes [n, 4, n_obs]."""
    dev = ctx.device
    n = _rows(stokes)
    params = torch.empty((n, NPAR), device=dev, dtype=torch.float32)
    pol = torch.empty(n, device=dev, dtype=torch.float32)
    ctx._check(lib().vfisv_init_classical(ctx._h, inst._h, n,
                                          _ptr(stokes, torch.float32, dev, n * 4 * inst.n_obs,
                                               name="stokes"),
                                          _ptr(params, torch.float32, dev),
                                          _ptr(pol, torch.float32, dev), _stream(dev)),
               "vfisv_init_classical")
    return params, pol


def init_combined(ctx, inst, stokes, base, pol_threshold=0.06, out=None):
    """Starting models [n, 10] combining base (e.g. the network's) with the
    classical azimuth everywhere and the classical B, gamma below
    pol_threshold; also returns the polarisation levels [n].  out may be
    base (in place)."""
    dev = ctx.device
    n = _rows(stokes)
    params = out if out is not None else torch.empty((n, NPAR), device=dev,
                                                     dtype=torch.float32)
    pol = torch.empty(n, device=dev, dtype=torch.float32)
    ctx._check(lib().vfisv_init_combined(ctx._h, inst._h, n,
                                         _ptr(stokes, torch.float32, dev, n * 4 * inst.n_obs,
                                              name="stokes"),
                                         _ptr(base, torch.float32, dev, n * NPAR, name="base"),
                                         float(pol_threshold),
                                         _ptr(params, torch.float32, dev, n * NPAR, name="out"),
                                         _ptr(pol, torch.float32, dev), _stream(dev)),
               "vfisv_init_combined")
    return params, pol


def autotune(ctx, inst, stokes, W, opts=None, sample=0):
    """Pick the derivative-pass split, persistent grid and pixel-queue block
    for this instrument's layout by timing them on the first ``sample``
    pixels; later inversions with automatic scheduling options use the
    choice.  Returns a dict."""
    dev = ctx.device
    o = (opts or Options()).c()
    t = _Tuning()
    n = _rows(stokes)
    ctx._check(lib().vfisv_autotune(
        ctx._h, inst._h, n, _ptr(stokes, torch.float32, dev, n * 4 * inst.n_obs, name="stokes"),
        _ptr(W, torch.float32, dev, _w_numel(W, n, inst.n_obs), name="W"),
        1 if W.dim() == 3 else 0, ctypes.byref(o),
        int(sample), ctypes.byref(t), _stream(dev)), "vfisv_autotune")
    return {k: getattr(t, k) for k, _ in _Tuning._fields_}


def stokes_weights(ctx, inst, stokes, mu, sigma=(1e-3, 1e-3, 1e-3, 1e-3), out=None):
    """Per-pixel weights W [n, 4, n_obs] of Eqs. 14-15 (w_I from the
    pixel's continuum against the centre-to-limb curve at mu [n]; Q, U, V
    weight one) divided by sigma^2 per Stokes parameter; pass the result to
    ``invert`` as W."""
    dev = ctx.device
    n = _rows(stokes)
    W = out if out is not None else torch.empty((n, 4, inst.n_obs), device=dev,
                                                dtype=torch.float32)
    sig = (ctypes.c_float * 4)(*[float(x) for x in sigma])
    ctx._check(lib().vfisv_stokes_weights(
        ctx._h, inst._h, n, _ptr(stokes, torch.float32, dev, n * 4 * inst.n_obs, name="stokes"),
        _ptr(mu, torch.float32, dev, n, name="mu"), sig,
        _ptr(W, torch.float32, dev, n * 4 * inst.n_obs, name="out"), _stream(dev)),
        "vfisv_stokes_weights")
    return W


def iter_histogram(ctx, iters, n_bins=51):
    """Histogram of iteration counts (device int32 tensor [n]) as a host
    numpy int64 array [n_bins]; the last bin counts iters >= n_bins - 1."""
    import numpy as np
    dev = ctx.device
    hist = np.zeros(n_bins, dtype=np.int64)
    n = _rows(iters, "iters")
    ctx._check(lib().vfisv_iter_histogram(
        ctx._h, n, _ptr(iters, torch.int32, dev, n, name="iters"), int(n_bins),
        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _stream(dev)),
        "vfisv_iter_histogram")
    return hist


def solve(ctx, H, g, eps, free_mask=0x3FF):
    """Damped solves: H [n, 55] float32 packed lower triangle, g [n, 10]
    float32, eps [n] float64 -> (delta [n, 10] float64, code [n] int32)."""
    dev = ctx.device
    n = _rows(H, "H")
    delta = torch.empty((n, NPAR), device=dev, dtype=torch.float64)
    code = torch.empty(n, device=dev, dtype=torch.int32)
    ctx._check(lib().vfisv_solve(ctx._h, n, _ptr(H, torch.float32, dev, n * 55, name="H"),
                                 _ptr(g, torch.float32, dev, n * NPAR, name="g"),
                                 _ptr(eps, torch.float64, dev, n, name="eps"), free_mask,
                                 _ptr(delta, torch.float64, dev, name="delta"),
                                 _ptr(code, torch.int32, dev, name="code"), _stream(dev)),
               "vfisv_solve")
    return delta, code

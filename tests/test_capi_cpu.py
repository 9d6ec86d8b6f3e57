"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/vfisv.h, and its host-side argument handling works."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_0901_2702_amd as vf
    if not os.path.exists(vf.LIB_PATH):
        from paper_0901_2702_amd import _build
        _build.build()
    return vf, vf.lib()


def _declared():
    src = open(os.path.join(ROOT, "include", "vfisv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vfisv_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("vfisv_create", "vfisv_destroy", "vfisv_instrument_create",
                     "vfisv_synthesize", "vfisv_invert", "vfisv_solve"):
        assert required in names


def test_every_declared_symbol_is_exported():
    vf, L = _lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(vf.EXPORTS)


def test_options_default_and_version():
    vf, L = _lib()
    o = vf._Options()
    L.vfisv_options_default(ctypes.byref(o))
    assert (o.max_iter, o.eps0, o.eps_max, o.rel_tol, o.free_mask, o.grid_waves,
            o.chunk_log2, o.lanes_per_pixel, o.voigt, o.fixed_iters, o.restarts,
            o.restart_seed, o.hess_reuse, o.fallback_rule, o.deriv_split) == (
        50, 1e-3, 1e8, 1e-5, 0x3FF, 0, -1, 1, 0, 0, 0, 0, 0.0, 0, -1)
    # the Python defaults are the library's
    d = vf.Options().c()
    assert all(getattr(d, f) == getattr(o, f) for f, _ in vf._Options._fields_)
    assert vf.version().startswith("vfisv-gfx950")


def test_null_arguments_are_rejected():
    vf, L = _lib()
    assert L.vfisv_create(None, 0) == -1
    assert b"NULL" in L.vfisv_last_error(None)
    assert L.vfisv_destroy(None) == 0
    assert L.vfisv_invert(None, None, 0, None, None, 0, None, None, None, None, None, None,
                          None) == -1
    assert L.vfisv_synthesize(None, None, 0, None, None, None, None, None) == -1
    assert L.vfisv_synthesize_voigt(None, None, 0, None, None, None, None, 0, None) == -1
    assert L.vfisv_solve(None, 0, None, None, None, 0, None, None, None) == -1
    assert L.vfisv_iter_histogram(None, 0, None, 1, None, None) == -1
    assert L.vfisv_autotune(None, None, 0, None, None, 0, None, 0, None, None) == -1
    assert L.vfisv_init_classical(None, None, 0, None, None, None, None) == -1
    assert L.vfisv_init_combined(None, None, 0, None, None, 0.06, None, None, None) == -1
    assert L.vfisv_stokes_weights(None, None, 0, None, None, None, None, None) == -1
    assert L.vfisv_instrument_info_get(None, None) == -1
    from paper_0901_2702_amd import learned
    L = learned._L()  # the network functions' signatures
    assert L.vfisv_mlp_num_inputs(None) == -1 and L.vfisv_mlp_num_params(None) == -1
    assert L.vfisv_mlp_stats(None, 0, 0, None, None, None, None, None, None, None) == -1
    assert L.vfisv_mlp_train(None, None, None, None, None, None, None) == -1
    assert L.vfisv_invert_learned(None, None, None, 0, None, None, 0, None, 0, 0.0, None, None,
                                  None, None, None) == -1


def test_no_cpu_fallback():
    """Without a HIP device the binding refuses to run rather than compute on
    the CPU."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    vf, _ = _lib()
    with pytest.raises(vf.VfisvError):
        vf.Context(0)


def test_binding_checks_sizes_before_any_call():
    """The library takes bare pointers; the binding refuses tensors whose
    element count, dtype or layout does not match what the call implies."""
    import torch
    from paper_0901_2702_amd import _ptr
    cpu = torch.device("cpu")
    t = torch.zeros((4, 10), dtype=torch.float32)
    assert _ptr(t, torch.float32, cpu, 40) == t.data_ptr()
    with pytest.raises(ValueError):
        _ptr(t, torch.float32, cpu, 41)
    with pytest.raises(TypeError):
        _ptr(t, torch.float64, cpu, 40)
    with pytest.raises(ValueError):
        _ptr(t.t(), torch.float32, cpu, 40)
    assert _ptr(None, torch.float32, cpu, 40) is None


def test_chi2_quantile_host_function():
    """The learned path's default threshold: the 0.99 quantile of
    chi^2_dof / dof, against the even-dof closed form (a Poisson sum) and
    against scipy for odd dof; bad arguments are refused."""
    import math
    from scipy.stats import chi2
    vf, L = _lib()
    L.vfisv_chi2_quantile.argtypes = [ctypes.c_int, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)]

    def q(k, p=0.99):
        out = ctypes.c_double()
        assert L.vfisv_chi2_quantile(k, p, ctypes.byref(out)) == 0
        return out.value

    def cdf_even(x, k):
        # 1 - exp(-x/2) sum_{j < k/2} (x/2)^j / j!, each term in log space
        h = 0.5 * x
        return 1.0 - sum(math.exp(j * math.log(h) - math.lgamma(j + 1) - h)
                         for j in range(k // 2))

    for k in (2, 14, 438, 4096):
        x = q(k) * k
        assert cdf_even(x, k) == pytest.approx(0.99, abs=1e-12), k
    for k in (1, 3, 15, 439):
        assert q(k) == pytest.approx(chi2.ppf(0.99, k) / k, rel=1e-12), k
    assert q(14, 0.5) == pytest.approx(chi2.ppf(0.5, 14) / 14, rel=1e-12)
    out = ctypes.c_double()
    assert L.vfisv_chi2_quantile(0, 0.99, ctypes.byref(out)) == -1
    assert L.vfisv_chi2_quantile(14, 1.0, ctypes.byref(out)) == -1
    assert L.vfisv_chi2_quantile(14, 0.99, None) == -1

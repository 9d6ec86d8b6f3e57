"""Sanitizer builds on the CPU: the FP64 oracle under AddressSanitizer +
UndefinedBehaviorSanitizer (plain and with its operation counters) and
under ThreadSanitizer (its thread pool), and the C-ABI library with its
host code under AddressSanitizer + UndefinedBehaviorSanitizer, driven
through every entry point that needs no GPU (tests/sanitize/*.c).  The
library's chi^2 quantile, computed on the host, is checked against scipy
over its whole domain on the way.

The sanitized library is built once per source state (about 90 s, device
code included) into paper_0901_2702_amd/_build/san/."""
import hashlib
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
SAN = os.path.join(ROOT, "tests", "sanitize")
PKG = os.path.join(ROOT, "paper_0901_2702_amd")
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build", "san")
ORACLE_SRCS = [os.path.join(ORACLE, s) for s in ("faddeeva.c", "me_forward.c", "lm.c")]
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
# host code only: each sanitizer flag applies to the host compilation
HOST_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-sanitize-recover=all -Xarch_host -fno-omit-frame-pointer").split()
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
           TSAN_OPTIONS="halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-6000:])
    return r


def _oracle_driver(tag, flags):
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver_" + tag)
    _run(["gcc", "-std=c11", "-O1", "-g", "-I", ORACLE] + flags
         + [os.path.join(SAN, "oracle_driver.c")] + ORACLE_SRCS + ["-lm", "-lpthread", "-o", exe])
    return exe


needs_gcc = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")


@needs_gcc
def test_oracle_under_address_and_undefined_sanitizers():
    exe = _oracle_driver("asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                  "-fno-omit-frame-pointer"])
    r = _run([exe, "4"], env=ENV, timeout=300)
    assert "oracle driver: ok" in r.stdout


@needs_gcc
def test_oracle_census_build_under_address_and_undefined_sanitizers():
    # the counters are not atomic: the census build runs on one thread
    exe = _oracle_driver("census_asan", ["-DORC_CENSUS", "-fsanitize=address,undefined",
                                         "-fno-sanitize-recover=all"])
    r = _run([exe, "1"], env=ENV, timeout=300)
    assert "oracle driver: ok" in r.stdout


@needs_gcc
def test_oracle_thread_pool_under_thread_sanitizer():
    exe = _oracle_driver("tsan", ["-fsanitize=thread"])
    r = _run([exe, "6"], env=ENV, timeout=300)
    assert "oracle driver: ok" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr


def _sanitized_library():
    srcs = ["kernels.hip", "capi.hip", "mlp.hip", "mlp_capi.hip", "classical.hip"]
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)) + ["../../include/vfisv.h"]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    h.update(" ".join(HOST_SAN).encode())
    lib = os.path.join(OUT, "libvfisv_san_%s.so" % h.hexdigest()[:16])
    if os.path.exists(lib):
        return lib
    os.makedirs(OUT, exist_ok=True)
    procs, objs = [], []
    for s in srcs:
        obj = os.path.join(OUT, s.replace(".hip", ".san.o"))
        cmd = ([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wno-unused-command-line-argument", "-Wno-unused-value"] + HOST_SAN
               + ["-I", CSRC, "-I", os.path.join(ROOT, "include"), "-c",
                  os.path.join(CSRC, s), "-o", obj])
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                       text=True), cmd))
        objs.append(obj)
    for p, cmd in procs:
        _, err = p.communicate()
        assert p.returncode == 0, "%s\n%s" % (" ".join(cmd), err[-4000:])
    tmp = lib + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + HOST_SAN[:4] + objs
         + ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-o", tmp])
    os.replace(tmp, lib)
    for f in os.listdir(OUT):  # builds of earlier source states
        if f.startswith("libvfisv_san_") and f.endswith(".so") and f != os.path.basename(lib):
            os.remove(os.path.join(OUT, f))
    return lib


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="ROCm compilers not found")
def test_c_abi_host_code_under_address_and_undefined_sanitizers():
    lib = _sanitized_library()
    exe = os.path.join(OUT, "capi_driver")
    _run([CLANG, "-std=c11", "-O1", "-g"] + HOST_SAN[:6]
         + ["-I", os.path.join(ROOT, "include"), os.path.join(SAN, "capi_driver.c"), lib,
            "-Wl,-rpath," + OUT, "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "capi driver: ok" in r.stdout
    from scipy.stats import chi2
    rows = [line.split()[1:] for line in r.stdout.splitlines() if line.startswith("quantile ")]
    assert len(rows) == 45
    for dof, q, x in rows:
        dof, q, x = int(dof), float(q), float(x)
        ref = chi2.ppf(q, dof) / dof
        np.testing.assert_allclose(x, ref, rtol=1e-9, err_msg="dof %d q %g" % (dof, q))

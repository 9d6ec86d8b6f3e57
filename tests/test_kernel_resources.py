"""Register budget of the inversion kernels, read from the compiler's own
resource report for gfx950 (no GPU needed).  The persistent LM kernels run
one wave per SIMD with every per-lane value in registers; an array that the
compiler cannot keep in registers goes to scratch memory and slows the
kernel many times over, so the only scratch allowed is the frame of the
eigen fallback (96 bytes per lane).  The device code also holds no packed
float32 arithmetic, on which the executed-FLOP figures from the hardware
counters rely."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0901_2702_amd", "csrc")


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


DEVICE_SOURCES = ("kernels.hip", "mlp.hip", "classical.hip", "capi.hip", "mlp_capi.hip")


@pytest.fixture(scope="module")
def device_asm(tmp_path_factory):
    """AMD assembly of every device source of the library for gfx950, built
    with the library's flags (in parallel)."""
    from paper_0901_2702_amd import _build
    d = tmp_path_factory.mktemp("asm")
    procs = {}
    for src in DEVICE_SOURCES:
        cmd = ([_hipcc()] + _build.HIPCC_FLAGS + ["-I", CSRC, "-I", os.path.join(ROOT, "include"),
               "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", str(d / (src + ".s"))])
        procs[src] = subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE)
    for src, p in procs.items():
        _, err = p.communicate()
        assert p.returncode == 0, (src, err[-2000:])
    return {src: (d / (src + ".s")).read_text() for src in DEVICE_SOURCES}


@pytest.fixture(scope="module")
def report(device_asm):
    text = device_asm["kernels.hip"]
    res = {}
    for m in re.finditer(r"^(_ZN5vfisv\w+):", text, re.M):
        seg = text[m.end():]
        get = lambda k: int(re.search(r"; %s: (\d+)" % k, seg).group(1))
        res[m.group(1)] = {k: get(k) for k in ("NumVgprs", "NumAgprs", "ScratchSize",
                                               "LDSByteSize")}
    return res


def test_lm_kernels_keep_their_state_in_registers(report):
    lm = {k: v for k, v in report.items() if "lm_kernel" in k or "lm_batches_kernel" in k}
    assert len(lm) >= 9
    for name, r in lm.items():
        assert r["ScratchSize"] <= 96, (name, r)
        assert r["NumVgprs"] <= 256, (name, r)
        # four one-wave workgroups per CU share its 160 KB of LDS
        assert 4 * r["LDSByteSize"] <= 160 * 1024, (name, r)


def test_synthesis_kernels_use_no_scratch(report):
    syn = {k: v for k, v in report.items() if "synth" in k}
    assert syn
    for name, r in syn.items():
        assert r["ScratchSize"] == 0, (name, r)


def test_no_packed_float32_arithmetic(device_asm):
    """The executed-FLOP figures count 2 per FMA and 1 per MUL, ADD or
    transcendental float32 instruction and lane: right only if no packed
    float32 instruction (two operations per lane, counted once by the SQ
    counters) is in the code, which the build's -packed-fp32-ops ensures."""
    packed = re.compile(r"^\s*v_pk_(fma|mul|add)_f32\b", re.M)
    for src, text in device_asm.items():
        assert not packed.search(text), src
    # the scan reads real code: float32 FMAs in the LM kernels, MFMAs in the network's
    assert re.search(r"^\s*v_fma_f32\b", device_asm["kernels.hip"], re.M)
    assert re.search(r"^\s*v_mfma_f32_16x16x32_bf16\b", device_asm["mlp.hip"], re.M)

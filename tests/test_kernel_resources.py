"""Register budget of the inversion kernels, read from the compiler's own
resource report for gfx950 (no GPU needed).  The persistent LM kernels run
one wave per SIMD with every per-lane value in registers; an array that the
compiler cannot keep in registers goes to scratch memory and slows the
kernel many times over, so the only scratch allowed is the frame of the
eigen fallback (96 bytes per lane)."""
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


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    from paper_0901_2702_amd import _build
    out = tmp_path_factory.mktemp("asm") / "kernels.s"
    cmd = ([_hipcc()] + _build.HIPCC_FLAGS + ["-I", CSRC, "-I", os.path.join(ROOT, "include"),
           "--cuda-device-only", "-S", os.path.join(CSRC, "kernels.hip"), "-o", str(out)])
    subprocess.run(cmd, check=True, capture_output=True)
    text = out.read_text()
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

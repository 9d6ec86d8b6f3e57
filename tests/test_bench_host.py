"""Host logic of bench.py (no GPU): the one-GPU contract, the census that
prices a launch's work, and the committed counter records it reads, which
must describe the kernel sources as they are."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as wl  # noqa: E402

PROFILES = os.path.join(ROOT, "profiles")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _census():
    info = {"n_active_fine": 59, "n_taps": 186}
    return bench.Census("hmi", info)


def test_census_prices_the_launch_counters():
    """float32 work = (trials + starts) x synthesis + Jacobians x (derivatives
    + normal equations); float64 work = (trials + starts) x chi^2 + trials x
    solve, with the per-unit counts of the committed census."""
    c = _census()
    work = {"pixels": 3, "trials": 10, "jacobians": 4}
    assert c.fp32(work) == pytest.approx(13 * c.trial + 4 * c.jac)
    assert c.fp64(work) == pytest.approx(13 * c.chi2 + 10 * c.solve)
    assert c.chi2 == 4 * 24 + 1  # Eq. 1 over the 24 residual rows
    rec = c.record()
    assert rec["fp32_per_trial"] == round(c.trial, 1)


def test_census_refuses_another_instrument():
    with pytest.raises(SystemExit):
        bench.Census("hmi", {"n_active_fine": 60, "n_taps": 186})


def test_the_census_instrument_is_the_benchmark_instrument():
    from oracle import census
    pts, _, taps = census.support(wl.hmi_instrument())
    assert (len(pts), taps) == (59, 186)


@pytest.mark.parametrize("profile", [bench.TRAFFIC_PROFILE, bench.LEARNED_TRAFFIC_PROFILE,
                                     bench.LEARNED_SQ_PROFILE, bench.FINE_TRAFFIC_PROFILE])
def test_committed_counter_records_describe_the_current_kernels(profile):
    """Each counter record names the kernel sources it was taken on; the
    benchmark reports its figures only while they match, and the committed
    records are kept current."""
    with open(profile) as fh:
        kv = dict(line.strip("- `\n").split(": ", 1) for line in fh
                  if line.startswith("- `") and ": " in line)
    assert kv["kernel_source_sha256"] == bench.kernel_source_hash(), os.path.basename(profile)
    n = int(kv["pixels"])
    if profile == bench.LEARNED_SQ_PROFILE:
        vals = bench.committed_values(profile, n)
        assert vals and vals["short_fit"] > 0 and vals["refit"] > 0
        assert vals["short_fit_trials"] > 0 and vals["refit_trials"] > 0
        assert bench.committed_values(profile, n + 1) is None
    else:
        t = bench.committed_traffic(n, profile)
        assert t and t["fetch_bytes"] > 0 and t["write_bytes"] > 0
        assert bench.committed_traffic(n + 1, profile) is None

"""Operation census of the inversion, counted by the oracle -- TEST INFRASTRUCTURE.

The oracle built with its operation counters (``liboracle_census.so``: the
same C sources with ORC_CENSUS defined; oracle.h lists the categories) runs
the LM fit of Sect. 4.2 with derivatives only after a successful trial
(Sect. 4.4, Fig. 6) on a sample of pixels of each instrument, and its
counters give the work of each unit of the method:

* one synthesis of the observed samples, values only (the trial of an LM
  iteration; Sect. 2, Eqs. 7-9, the filters of Sect. 5), with H and F taken
  from the second-order Taylor table of Sect. 3.2 (Eqs. 10-13), the
  evaluation the paper uses;
* the derivatives of that synthesis with respect to the ten parameters
  (forward mode, only the components that are not identically zero), done
  once per start and per accepted model;
* the normal equations J^T W J (one triangle) and J^T W r of Eqs. 2-4;
* chi^2 of Eq. 1, once per synthesis;
* the damped solve of Eq. 5 and the step.

One count per +, -, * or / on a double (sqrt, sin, cos and rounding are
listed apart).  The census instrument keeps the filter taps at or above
2^-24 of their row's largest (a smaller tap changes no float32 sample) and
the synthesis points that some kept tap reads.

    python -m oracle.census [--out profiles/flop_census.md]

writes the table and a machine-readable record per instrument
(``- `hmi.<key>: value` ``) that the benchmark reads.
"""
import argparse
import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import build as _build  # noqa: E402
import workloads as wl  # noqa: E402

CATEGORIES = ("value", "gradient", "voigt_calls", "voigt", "chi2", "normal", "solve",
              "special")
TAP_FLOOR = 2.0 ** -24
SEED = 1000  # the 64 x 64 HMI set's priors and noise stream

_CLIB = None


def census_lib():
    global _CLIB
    if _CLIB is None:
        _build.build_census()
        L = oracle.bind(_build.CENSUS_LIB)
        L.orc_census_take.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        L.orc_census_take.restype = None
        _CLIB = L
    return _CLIB


def take():
    out = (ctypes.c_uint64 * len(CATEGORIES))()
    census_lib().orc_census_take(out)
    return dict(zip(CATEGORIES, (int(x) for x in out)))


def support(spec):
    """The kept taps and the synthesis points they read: (point indices,
    filter restricted to them, number of kept taps)."""
    F = np.asarray(spec.filter, dtype=np.float64)
    keep = (F > 0.0) & (F >= TAP_FLOOR * F.max(axis=1, keepdims=True))
    Fk = np.where(keep, F, 0.0)
    pts = np.nonzero(keep.any(axis=0))[0]
    return pts, Fk[:, pts], int(keep.sum())


def census(spec, n_pixels, seed=SEED):
    """Per-unit operation counts of the method on one instrument."""
    pts, Fk, n_taps = support(spec)
    ci = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA[pts], Fk, voigt=2)
    exact = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    P = wl.draw_params(n_pixels, seed)
    obs = (oracle.forward_batch(exact, P) + wl.draw_noise(n_pixels, spec.n_obs, seed)
           ).astype(np.float32)
    W = wl.weights(spec.n_obs)
    L = census_lib()
    take()
    # one synthesis, values only and with derivatives, at each pixel's model
    S = np.empty((4, spec.n_obs))
    J = np.empty((4, spec.n_obs, oracle.NPAR))
    vals, grads, voigts = [], [], []
    for p in P:
        m = np.ascontiguousarray(p)
        L.orc_forward(ctypes.byref(ci.c), oracle._d(m), oracle._d(S), None)
        v = take()
        L.orc_forward(ctypes.byref(ci.c), oracle._d(m), oracle._d(S), oracle._d(J))
        g = take()
        assert v["voigt_calls"] == g["voigt_calls"] == 3 * len(pts)
        assert g["value"] == v["value"] and g["voigt"] == v["voigt"]
        vals.append(v["value"] + v["voigt"])
        voigts.append(v["voigt"] / v["voigt_calls"])
        grads.append(g["gradient"])
    # whole fits from the default model: chi^2, normal equations and solves
    tot = dict.fromkeys(CATEGORIES, 0)
    calls = dict(trials=0, derivs=0, solves=0, hessians=0)
    for i in range(n_pixels):
        r = _lm_pixel(L, ci, obs[i], W)
        c = take()
        for k in CATEGORIES:
            tot[k] += c[k]
        for k in calls:
            calls[k] += r[k]
    assert calls["hessians"] == calls["derivs"]
    rows = 4 * spec.n_obs
    out = dict(points=len(pts), taps=n_taps, rows=rows, pixels=n_pixels,
               synthesis_values=float(np.mean(vals)),
               synthesis_values_min=int(np.min(vals)), synthesis_values_max=int(np.max(vals)),
               voigt_per_evaluation=float(np.mean(voigts)),
               synthesis_derivatives=float(np.mean(grads)),
               normal_equations=tot["normal"] / calls["derivs"],
               chi2=tot["chi2"] / (calls["trials"] + calls["derivs"]),
               solve=tot["solve"] / calls["solves"],
               trials=calls["trials"], jacobians=calls["derivs"])
    assert out["chi2"] == 4 * rows + 1
    return out


def _lm_pixel(L, ci, obs, W):
    opts = oracle.Options().c()
    M = np.empty(oracle.NPAR)
    chi2 = np.empty(1)
    it = np.empty(1, np.int32)
    st = np.empty(1, np.int32)
    cnt = oracle._Counters()
    o = np.ascontiguousarray(obs)
    w = np.ascontiguousarray(W)
    L.orc_lm_pixel(ctypes.byref(ci.c), ctypes.byref(opts), oracle._f(o), oracle._f(w), None, 0,
                   oracle._d(M), oracle._d(chi2), oracle._i(it), oracle._i(st),
                   ctypes.byref(cnt))
    return dict(trials=cnt.trials, derivs=cnt.derivs, solves=cnt.solves, hessians=cnt.hessians)


KEYS = ("points", "taps", "synthesis_values", "synthesis_derivatives", "normal_equations",
        "chi2", "solve", "voigt_per_evaluation")


def report(results):
    lines = ["# Operation census of the inversion, counted by the oracle", "",
             "Command (from the repository root): `python -m oracle.census`", "",
             "The oracle built with ORC_CENSUS counts one operation per +, -, * or / on a "
             "double as it runs (sqrt, sin, cos and rounding apart).  Synthesis with H and F "
             "from the second-order Taylor table (Sect. 3.2, Eqs. 10-13); derivatives in "
             "forward mode over the components that are not identically zero; one triangle "
             "of J^T W J.  Filter taps at or above 2^-24 of their row's largest and the "
             "synthesis points they read.  Per-synthesis counts are averaged over the "
             "pixels' true models; chi^2, normal equations and solves over whole fits from "
             "the default model (Sect. 4.2, derivatives only after success, Fig. 6).", "",
             "| Unit | " + " | ".join(results) + " |",
             "|---|" + "---|" * len(results)]
    rows = [("synthesis points / kept taps / residual rows",
             lambda r: "%d / %d / %d" % (r["points"], r["taps"], r["rows"])),
            ("synthesis, values (one trial)", lambda r: "%.1f (%d..%d)" % (
                r["synthesis_values"], r["synthesis_values_min"], r["synthesis_values_max"])),
            ("  of which per H, F evaluation (3 per point)",
             lambda r: "%.2f" % r["voigt_per_evaluation"]),
            ("synthesis, derivatives (per start or accepted model)",
             lambda r: "%.1f" % r["synthesis_derivatives"]),
            ("normal equations (per start or accepted model)",
             lambda r: "%.1f" % r["normal_equations"]),
            ("chi^2 (per synthesis)", lambda r: "%.0f" % r["chi2"]),
            ("damped solve and step (per trial)", lambda r: "%.1f" % r["solve"]),
            ("sample: pixels, trials, Jacobians",
             lambda r: "%d, %d, %d" % (r["pixels"], r["trials"], r["jacobians"]))]
    for name, f in rows:
        lines.append("| %s | " % name + " | ".join(f(r) for r in results.values()) + " |")
    lines += ["", "Machine-readable record:", ""]
    for inst, r in results.items():
        for k in KEYS:
            v = r[k]
            lines.append("- `%s.%s: %s`" % (inst, k, ("%d" % v) if isinstance(v, int)
                                             else ("%.4f" % v)))
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "flop_census.md"))
    ap.add_argument("--hmi-pixels", type=int, default=64)
    ap.add_argument("--fine-pixels", type=int, default=8)
    args = ap.parse_args()
    res = {"hmi": census(wl.hmi_instrument(), args.hmi_pixels),
           "fine": census(wl.fine_instrument(), args.fine_pixels)}
    text = report(res)
    with open(args.out, "w") as fh:
        fh.write(text)
    print(text)


if __name__ == "__main__":
    main()

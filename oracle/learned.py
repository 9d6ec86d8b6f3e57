"""FP64 oracle of the learned-start inversion and its fallback -- TEST
INFRASTRUCTURE (only the tests, the smoke check and the benchmark's CPU
baseline may use it).

Sect. 5 of the paper starts the inversion from a network's guess (with the
weak-field and azimuth estimates as a second initialisation) and asks that
the guess cost only a small fraction of the inversion; it does not say what
is done for pixels the guess serves badly.  The path the library implements,
step by step in the order it runs:

1. the network's starting model of every pixel: the standardised samples
   through the network (``mlp.forward``), the ten codes decoded
   (``mlp.decode_outputs``), the result projected into the parameter box;
2. Levenberg-Marquardt from that model with at most ``short_max_iter``
   (15) trials (the oracle's LM, ``oracle.invert``);
3. the pixels whose reduced chi^2 (Eq. 1) then exceeds tau are fitted again
   with the full trial budget (50) from the combined start of Sect. 5: the
   network's model with the classical azimuth, and with the weak-field B
   and inclination where the polarisation level is below 6%
   (``classical.combined_init``); tau defaults to the 0.99 quantile of
   chi^2_dof / dof, which a pixel fitted down to its noise stays below with
   probability 0.99;
4. of the two fits the one with the lower chi^2 is kept; iters counts the
   trials of both fits, and the status gets the FALLBACK bit (16).
Pixels with non-finite samples end NONFINITE after step 2 and are not
fitted again.

``rule`` switches the three choices of steps 3-4 to the fallback as first
stated for this path: REFIT_UNCONVERGED also re-fits pixels whose short fit
did not converge, REFIT_FROM_DEFAULT starts the re-fit from the default
model, REFIT_KEEP_REFIT keeps the re-fit even where it is worse.
"""
import numpy as np
from scipy.stats import chi2 as _chi2

import oracle
from . import classical
from . import mlp

FALLBACK = 16
REFIT_UNCONVERGED, REFIT_FROM_DEFAULT, REFIT_KEEP_REFIT = 1, 2, 4
AS_STATED = REFIT_UNCONVERGED | REFIT_FROM_DEFAULT | REFIT_KEEP_REFIT
HIDDEN = 256
CODE_PAD = 32


def reduced_chi2_quantile(dof, q=0.99):
    """q-quantile of chi^2_dof / dof (the default tau of step 3)."""
    return float(_chi2.ppf(q, dof) / dof)


def unpack_params(flat, n_in):
    """The network's float32 parameters in the library's packed order
    (W1 [K0][256] with K0 = n_in rounded up to 32, b1, W2, b2, W3, b3,
    W4 [256][32], b4 [32]) as float64 arrays for mlp.forward, with the
    zero padding of the first layer's inputs and of the outputs dropped."""
    K0 = (n_in + 31) // 32 * 32
    shapes = [(K0, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,),
              (HIDDEN, CODE_PAD), (CODE_PAD,)]
    flat = np.asarray(flat)
    out, off = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        out.append(flat[off:off + k].reshape(sh).astype(np.float64))
        off += k
    if off != flat.size:
        raise ValueError("parameter vector of %d values, expected %d" % (flat.size, off))
    return {"W1": out[0][:n_in], "b1": out[1], "W2": out[2], "b2": out[3], "W3": out[4],
            "b3": out[5], "W4": out[6][:, :10], "b4": out[7][:10]}


def standardise(samples, in_mean, in_std):
    """(x - mean) / std as the network's input layer takes it: float32
    difference times the float32 reciprocal of std."""
    x = np.asarray(samples, dtype=np.float32)
    m = np.asarray(in_mean, dtype=np.float32)
    r = (np.float32(1.0) / np.asarray(in_std, dtype=np.float32)).astype(np.float32)
    return ((x - m) * r).astype(np.float32)


def network_starts(flat, n_in, in_mean, in_std, out_mean, out_std, samples, emulate_bf16=True):
    """Step 1: starting models [n, 10] (and the codes [n, 10]) of the pixels
    samples [n, n_in] from the network with parameters flat."""
    P = unpack_params(flat, n_in)
    xs = standardise(np.asarray(samples).reshape(-1, n_in), in_mean, in_std)
    y, _ = mlp.forward(P, xs, emulate_bf16=emulate_bf16)
    M = mlp.decode_outputs(y, np.asarray(out_mean, np.float64), np.asarray(out_std, np.float64))
    return np.array([oracle.project(m) for m in M]), y


def combined_starts(inst, obs, base, pol_threshold=0.06):
    """The combined start of Sect. 5 over the pixels obs [n, 4, n_obs]."""
    x = classical.sample_offsets(inst.filt, inst.fine)
    cz = oracle.zeeman_constant(inst.lambda0_A, inst.geff)
    M, _ = classical.combined_init(obs, base, pol_threshold, x, inst.lambda0_A, cz,
                                   oracle.default_init(), oracle.project)
    return M


def learned_invert(inst, obs, W, starts, opts=None, short_max_iter=15, tau=None, rule=0,
                   pol_threshold=0.06, nthreads=0):
    """Steps 2-4 from the starting models starts [n, 10].

    obs [n, 4, n_obs] float32; W [4, n_obs] or [n, 4, n_obs]; opts: the
    oracle's LM options of the re-fit (its max_iter is the full budget).
    Returns dict(params, chi2, iters, status, refit (bool [n]), short (the
    short fit's dict), tau)."""
    opts = opts or oracle.Options()
    obs = np.ascontiguousarray(obs, dtype=np.float32)
    n = obs.shape[0]
    W = np.ascontiguousarray(W, dtype=np.float32)
    per_pixel = W.ndim == 3
    nfree = bin(opts.free_mask & 0x3FF).count("1")
    dof = 4 * inst.n_obs - nfree
    if tau is None:
        tau = reduced_chi2_quantile(dof)
    so = oracle.Options(**{**opts.__dict__, "max_iter": short_max_iter})
    short = oracle.invert(inst, obs, W, init=starts, opts=so, nthreads=nthreads)
    c = short["chi2"]
    code = short["status"] & 15
    finite = ~np.isnan(c)
    refit = finite & ~(c <= tau)
    if rule & REFIT_UNCONVERGED:
        refit |= finite & (code != oracle.CONVERGED) & (code != oracle.NONFINITE)
    out = {k: np.array(short[k]) for k in ("params", "chi2", "iters", "status")}
    idx = np.flatnonzero(refit)
    if idx.size:
        sub = obs[idx]
        if rule & REFIT_FROM_DEFAULT or inst.n_obs < 3:
            start = None
        else:
            start = combined_starts(inst, sub, np.asarray(starts, np.float64)[idx], pol_threshold)
        r = oracle.invert(inst, sub, W[idx] if per_pixel else W, init=start, opts=opts,
                          nthreads=nthreads)
        take = np.ones(idx.size, bool) if rule & REFIT_KEEP_REFIT else r["chi2"] < c[idx]
        out["params"][idx[take]] = r["params"][take]
        out["chi2"][idx[take]] = r["chi2"][take]
        out["status"][idx[take]] = r["status"][take]
        out["iters"][idx] += r["iters"]
        out["status"][idx] |= FALLBACK
    out.update(refit=refit, short=short, tau=tau)
    return out

"""Classical initial guess on the GPU against the FP64 oracle (Sect. 5:
weak-field B and gamma, linear-polarisation azimuth, line position), for the
HMI-shaped and the fine-spectrum instruments, on oracle-made observations."""
import numpy as np
import pytest
import torch

import oracle
from oracle import classical
import workloads as wl

pytestmark = pytest.mark.gpu

vf = pytest.importorskip("paper_0901_2702_amd")


@pytest.fixture(scope="module")
def ctx():
    print("[gpu-classical] creating context", flush=True)
    return vf.Context(0)


U32 = 2.0 ** -24  # unit roundoff of float32
C_KMS = classical.C_KMS
ALPHA0 = classical.ALPHA0


def _within_f32_bounds(which, d, bounds):
    """Every pixel's difference within twice its first-order bound (the
    factor covers second-order terms and the float64 functions' own few
    ulps); prints how close the largest differences come."""
    names = ("B", "gamma", "psi", "v")
    for j, k in enumerate(names[:d.shape[1]]):
        bnd = bounds[k]
        chk = np.isfinite(bnd)
        ratio = d[chk, j] / np.maximum(bnd[chk], 1e-300)
        print("[gpu-classical] %s %s: %d pixels bounded, max |d| / bound %.3f, median bound %.2e"
              % (which, k, chk.sum(), ratio.max(), np.median(bnd[chk])), flush=True)
        assert chk.mean() > 0.99, (which, k)
        assert np.all(d[chk, j] <= 2.0 * bnd[chk]), (which, k, ratio.max())


def _f32_bounds(obs, x, cz, lambda0_A):
    """Per-pixel first-order bounds on |GPU - oracle| for B [G], gamma and psi
    [deg] and v [km/s] when the sums of the classical estimates (the
    depression and its first moment, sum V I', sum I'^2, sum |Q + iU| |I''|,
    sum I''^2, sum U, sum Q) are accumulated in float32 from the same float32
    samples, in any order, and the rest is float64.  Standard rounding-error
    analysis (Higham, Accuracy and Stability of Numerical Algorithms, ch. 3):
    a float32 product or quotient carries a relative error u, a difference of
    float32 values u of its result, the sample offsets u of their value, and a
    sum of m terms at most (m - 1) u times the sum of the terms' magnitudes;
    the errors of the sums then propagate through the float64 formulas by
    their partial derivatives.  Each output is rounded to float32 (u more)."""
    S = np.asarray(obs, dtype=np.float64)
    I, Q, U, V = S[:, 0], S[:, 1], S[:, 2], S[:, 3]
    x = np.asarray(x, dtype=np.float64)
    no = x.size
    u = U32
    acc = no * u  # accumulation over the samples

    def sum_err(terms, term_err):
        """|error| of a float32 sum whose terms carry term_err each."""
        return term_err.sum(axis=1) + acc * np.abs(terms).sum(axis=1)

    Ic = I.max(axis=1)
    d = Ic[:, None] - I
    sd, sdx = d.sum(axis=1), (d * x).sum(axis=1)
    e_sd = sum_err(d, u * np.abs(d))
    e_sdx = sum_err(d * x, 3 * u * np.abs(d * x))
    # first differences (central inside, one-sided at the ends)
    a = np.maximum(np.arange(no) - 1, 0)
    b = np.minimum(np.arange(no) + 1, no - 1)
    D = x[b] - x[a]
    Ip = (I[:, b] - I[:, a]) / D
    e_Ip = np.abs(Ip) * (3 * u + u * (np.abs(x[a]) + np.abs(x[b])) / np.abs(D))
    # second differences at the interior sample nearest k
    c = np.clip(np.arange(no), 1, no - 2)
    h0, h1 = x[c] - x[c - 1], x[c + 1] - x[c]
    e_h0 = u * (np.abs(x[c]) + np.abs(x[c - 1]) + np.abs(h0))
    e_h1 = u * (np.abs(x[c + 1]) + np.abs(x[c]) + np.abs(h1))
    t0, t1, t2 = h0 * I[:, c + 1], (h0 + h1) * I[:, c], h1 * I[:, c - 1]
    N = t0 - t1 + t2
    e_N = (e_h0 * np.abs(I[:, c + 1]) + (e_h0 + e_h1 + u * np.abs(h0 + h1)) * np.abs(I[:, c])
           + e_h1 * np.abs(I[:, c - 1]) + 3 * u * (np.abs(t0) + np.abs(t1) + np.abs(t2)))
    Dn = h0 * h1 * (h0 + h1)
    rel_Dn = (e_h0 / np.abs(h0) + e_h1 / np.abs(h1) + (e_h0 + e_h1) / np.abs(h0 + h1) + 3 * u)
    Ipp = 2.0 * N / Dn
    e_Ipp = 2.0 * e_N / np.abs(Dn) + np.abs(Ipp) * (rel_Dn + u)
    L = np.sqrt(Q * Q + U * U)
    e_L = 4 * u * L
    sVI, sII = (V * Ip).sum(axis=1), (Ip * Ip).sum(axis=1)
    e_sVI = sum_err(V * Ip, np.abs(V) * e_Ip + u * np.abs(V * Ip))
    e_sII = sum_err(Ip * Ip, 2 * np.abs(Ip) * e_Ip + u * Ip * Ip)
    sLI, sI2 = (L * np.abs(Ipp)).sum(axis=1), (Ipp * Ipp).sum(axis=1)
    e_sLI = sum_err(L * np.abs(Ipp), e_L * np.abs(Ipp) + L * e_Ipp + u * L * np.abs(Ipp))
    e_sI2 = sum_err(Ipp * Ipp, 2 * np.abs(Ipp) * e_Ipp + u * Ipp * Ipp)
    sU, sQ = U.sum(axis=1), Q.sum(axis=1)
    e_sU, e_sQ = acc * np.abs(U).sum(axis=1), acc * np.abs(Q).sum(axis=1)
    # float64 from here on, with the constants rounded to float32 (u each)
    with np.errstate(divide="ignore", invalid="ignore"):
        lam = sdx / sd
        e_lam = np.abs(e_sdx / sd) + np.abs(sdx) * e_sd / sd ** 2
        v = C_KMS * lam / (lambda0_A * 1000.0)
        e_v = C_KMS / (lambda0_A * 1000.0) * e_lam + 4 * u * np.abs(v)
        b_par = -sVI / (cz * sII)
        e_bpar = (e_sVI + np.abs(sVI) * e_sII / sII) / (cz * sII) + u * np.abs(b_par)
        bp2 = 4.0 * sLI / (cz * cz * sI2)
        e_bp2 = 4.0 * (e_sLI + sLI * e_sI2 / sI2) / (cz * cz * sI2) + 3 * u * np.abs(bp2)
        bl = b_par / ALPHA0
        bt = np.sqrt(np.maximum(bp2, 0.0) / ALPHA0)
        e_bl = e_bpar / ALPHA0
        # |sqrt(a + e) - sqrt(a)| <= min(e / (2 sqrt(a)), sqrt(e))
        e_bt = np.minimum(e_bp2 / ALPHA0 / (2.0 * bt), np.sqrt(e_bp2 / ALPHA0))
        B = np.hypot(bl, bt)
        e_B = e_bl + e_bt + u * B
        e_g = np.degrees((np.abs(bl) * e_bt + bt * e_bl) / B ** 2) + u * 180.0
        e_psi = np.degrees(0.5 * (np.abs(sQ) * e_sU + np.abs(sU) * e_sQ) / (sQ ** 2 + sU ** 2)) \
            + u * 180.0
    # a vanishing sum is exact on both sides (all its terms vanish)
    e_bt = np.where(sI2 == 0, 0.0, e_bt)
    e_v = np.where(sd == 0, 0.0, e_v)
    e_B = np.where(sII == 0, e_bt + u * B, e_B)
    return dict(B=e_B, gamma=np.nan_to_num(e_g, nan=np.inf), psi=np.nan_to_num(e_psi, nan=np.inf),
                v=e_v)


@pytest.mark.parametrize("which", ["hmi", "fine"])
def test_classical_start_matches_the_oracle(ctx, which):
    spec = wl.hmi_instrument() if which == "hmi" else wl.fine_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    n = 4096 if which == "hmi" else 512
    P = wl.draw_params(n, 61)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, 61)).astype(np.float32)
    obs[:8] = oracle.forward_batch(oi, P[:8])  # a few noiseless pixels
    x = classical.sample_offsets(spec.filter, spec.fine_offset_mA)
    cz = oracle.zeeman_constant(spec.lambda0_A, spec.geff)
    ref, pol_ref = classical.classical_init(obs, x, spec.lambda0_A, cz, wl.default_model(),
                                            oracle.project)
    g, pol = vf.init_classical(ctx, inst, torch.tensor(obs, device=ctx.device))
    g, pol = g.cpu().numpy().astype(np.float64), pol.cpu().numpy()
    d = np.abs(g - ref)
    d[:, 2] = np.minimum(d[:, 2], 180.0 - d[:, 2])
    _within_f32_bounds(which, d, _f32_bounds(obs, x, cz, spec.lambda0_A))
    # S0, S1 = 0.3 I_c, 0.7 I_c with I_c a sample: only the output's rounding
    assert np.all(d[:, 7:9] <= U32 * np.abs(ref[:, 7:9]))
    np.testing.assert_array_equal(g[:, [4, 5, 6, 9]], ref[:, [4, 5, 6, 9]].astype(np.float32))
    np.testing.assert_allclose(pol, pol_ref, rtol=1e-4, atol=1e-9)
    # a buffer that is not 16-byte aligned takes the generic kernel
    flat = torch.zeros(obs.size + 1, device=ctx.device)
    flat[1:] = torch.tensor(obs.ravel(), device=ctx.device)
    gm, pm = vf.init_classical(ctx, inst, flat[1:].view(obs.shape))
    gm = gm.cpu().numpy().astype(np.float64)
    dm = np.abs(gm - g)
    dm[:, 2] = np.minimum(dm[:, 2], 180.0 - dm[:, 2])
    assert np.quantile(dm[:, 0] / np.maximum(g[:, 0], 1.0), 0.999) < 1e-5
    assert np.quantile(dm[:, 1:3], 0.999) < 1e-3 and dm[:, 3].max() < 1e-5
    np.testing.assert_array_equal(pm.cpu().numpy(), pol)
    # non-finite samples: default model, polarisation level NaN
    bad = obs[:4].copy()
    bad[1, 3, 2] = np.nan
    gb, pb = vf.init_classical(ctx, inst, torch.tensor(bad, device=ctx.device))
    np.testing.assert_array_equal(gb.cpu().numpy()[1], wl.default_model().astype(np.float32))
    assert np.isnan(pb.cpu().numpy()[1]) and np.isfinite(pb.cpu().numpy()[[0, 2, 3]]).all()


def test_combined_start_matches_the_oracle(ctx):
    """Network-style base models combined with the classical azimuth and,
    below 6 % polarisation, the classical B and gamma; in place and out of
    place give the same bits."""
    spec = wl.hmi_instrument()
    inst = vf.Instrument.from_spec(ctx, spec)
    oi = oracle.Instrument(spec.lambda0_A, spec.geff, spec.fine_offset_mA, spec.filter)
    n = 4096
    P = wl.draw_params(n, 62)
    obs = (oracle.forward_batch(oi, P) + wl.draw_noise(n, spec.n_obs, 62)).astype(np.float32)
    obs[5, 0, 1] = np.inf                      # keeps the base model
    obs[6] = -np.abs(obs[6])                   # no continuum: level NaN
    base = wl.draw_params(n, 63).astype(np.float32)
    x = classical.sample_offsets(spec.filter, spec.fine_offset_mA)
    cz = oracle.zeeman_constant(spec.lambda0_A, spec.geff)
    thr = 0.06
    ref, pol_ref = classical.combined_init(obs, base.astype(np.float64), thr, x, spec.lambda0_A,
                                           cz, wl.default_model(), oracle.project)
    dev = ctx.device
    tb = torch.tensor(base, device=dev)
    g, pol = vf.init_combined(ctx, inst, torch.tensor(obs, device=dev), tb, thr)
    g2, _ = vf.init_combined(ctx, inst, torch.tensor(obs, device=dev), tb.clone(), thr,
                             out=None)
    inplace = tb.clone()
    vf.init_combined(ctx, inst, torch.tensor(obs, device=dev), inplace, thr, out=inplace)
    assert torch.equal(g, g2) and torch.equal(g, inplace)
    g, pol = g.cpu().numpy().astype(np.float64), pol.cpu().numpy()
    assert np.isnan(pol[5]) and np.isnan(pol[6])
    # the selection is taken on the GPU's own float32 level; pixels whose
    # FP64 level lies within rounding of the threshold are left out
    low_gpu = pol < thr
    sure = ~np.isclose(pol_ref, thr, rtol=1e-4, atol=0) | np.isnan(pol_ref)
    assert np.array_equal(low_gpu[sure], (pol_ref < thr)[sure])
    assert 0.1 < low_gpu.mean() < 0.9
    d = np.abs(g - ref)
    d[:, 2] = np.minimum(d[:, 2], 180.0 - d[:, 2])
    with np.errstate(invalid="ignore"):  # the non-finite pixel's bounds are NaN
        bounds = _f32_bounds(obs, x, cz, spec.lambda0_A)
    print("[gpu-classical] combined: %.3f below threshold" % low_gpu.mean(), flush=True)
    fin = np.isfinite(obs).all(axis=(1, 2))
    low = sure & low_gpu & fin
    _within_f32_bounds("combined, low polarisation", d[low][:, :3],
                       {k: bounds[k][low] for k in ("B", "gamma", "psi")})
    # the azimuth is the classical one on every pixel with finite samples
    ok = sure & fin
    assert np.all(d[ok, 2] <= 2.0 * bounds["psi"][ok])
    # everything else is the base, bit for bit after the box
    np.testing.assert_array_equal(g[:, 3:], ref[:, 3:].astype(np.float32))
    np.testing.assert_array_equal(g[~low_gpu & sure, :2],
                                  ref[~low_gpu & sure, :2].astype(np.float32))
    np.testing.assert_array_equal(g[5], ref[5].astype(np.float32))

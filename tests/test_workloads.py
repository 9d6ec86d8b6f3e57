"""The synthetic input generators (numbers only, no method arithmetic)."""
import numpy as np

import workloads as wl


def test_disk_count_of_the_full_disk():
    # centre (2047.5, 2047.5), radius 2048 on a 4096 x 4096 grid
    assert int(wl.disk_mask(4096).sum()) == 13_176_792


def _image(mask, flag):
    img = np.zeros(mask.shape, dtype=bool)
    img[mask] = flag
    return img


def test_full_disk_split_ranges_and_clustering():
    for clustered in (True, False):
        P, active, mask = wl.full_disk(grid=512, seed=3, clustered=clustered)
        n = int(mask.sum())
        assert P.shape == (n, 10) and active.shape == (n,)
        frac = active.mean()
        if clustered:
            assert 0.2 <= frac < 0.23
        else:
            assert abs(frac - 0.2) < 0.01
        B = P[:, 0]
        assert (B[active] >= 500).all() and (B[active] <= 3500).all()
        assert (B[~active] >= 0).all() and (B[~active] <= 200).all()
        # the other parameters keep the synthetic priors
        assert (P[:, 4] >= 20).all() and (P[:, 4] <= 50).all()
        np.testing.assert_allclose(P[:, 7] + P[:, 8], 1.0)
        # neighbour of an active pixel is active: clustered >> i.i.d.
        img = _image(mask, active)
        both = img[:, :-1] & img[:, 1:] & mask[:, 1:]
        p_nb = both.sum() / (img[:, :-1] & mask[:, 1:]).sum()
        if clustered:
            assert p_nb > 0.9
        else:
            assert abs(p_nb - 0.2) < 0.02
    # seeded: the same call gives the same pixels, another seed does not
    a = wl.full_disk(grid=256, seed=9)
    b = wl.full_disk(grid=256, seed=9)
    c = wl.full_disk(grid=256, seed=10)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[1], c[1])


def test_disk_mu():
    mu = wl.disk_mu(64)
    assert mu.shape == (int(wl.disk_mask(64).sum()),)
    assert 0.0 <= mu.min() < 0.2 and 0.99 < mu.max() <= 1.0
    # the pixels with mu above m fill the disk area inside rho = sqrt(1 - m^2)
    m = 0.6
    assert abs(np.mean(mu > m) - (1 - m * m)) < 0.02

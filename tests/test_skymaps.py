"""Equal-area sky pixels and angular power used by the lightcone map comparison.

Pins: the twelve base pixels of the ring scheme sit at z = 2/3, 0, -2/3 with the published
azimuths (Gorski et al. 2005); pixel centres map back to their own pixels; uniform random
directions fill every pixel equally (equal areas); the power of a single spherical harmonic
lands at its own l with C_l = |a|^2 / (2 l + 1).
"""
import math

import numpy as np
import pytest
import torch

sk = pytest.importorskip("paper_2005_05328_amd.skymaps")


def test_base_pixels():
    z, phi = sk.ring_pix2ang(1, np.arange(12))
    assert np.allclose(z[:4], 2.0 / 3.0) and np.allclose(z[4:8], 0.0)
    assert np.allclose(z[8:], -2.0 / 3.0)
    assert np.allclose(phi[:4], [(2 * k + 1) * math.pi / 4 for k in range(4)])
    assert np.allclose(phi[4:8], [k * math.pi / 2 for k in range(4)])
    assert np.allclose(phi[8:], [(2 * k + 1) * math.pi / 4 for k in range(4)])


@pytest.mark.parametrize("nside", [1, 2, 8, 32])
def test_centres_round_trip(nside):
    npix = 12 * nside * nside
    z, phi = sk.ring_pix2ang(nside, np.arange(npix))
    assert np.array_equal(sk.ring_ang2pix(nside, z, phi), np.arange(npix))
    zt, pt = torch.from_numpy(z), torch.from_numpy(phi)
    assert np.array_equal(sk.ring_ang2pix(nside, zt, pt).numpy(), np.arange(npix))
    # rings: 4 nside - 1 distinct latitudes
    assert np.unique(np.round(z, 12)).size == 4 * nside - 1


def test_equal_areas():
    nside, n = 8, 3_000_000
    g = np.random.default_rng(5)
    v = g.standard_normal((n, 3))
    counts = np.asarray(sk.sky_map(torch.from_numpy(v), torch.ones(n, dtype=torch.float64),
                                   nside))
    npix = 12 * nside * nside
    mean = n / npix
    chi2 = float(((counts - mean) ** 2 / mean).sum())
    assert counts.sum() == n
    # chi-square with npix - 1 degrees of freedom: within 5 sigma of its mean
    assert abs(chi2 - (npix - 1)) < 5 * math.sqrt(2 * (npix - 1))


def test_single_harmonic_power():
    from scipy.special import sph_harm_y
    nside, ell = 32, 5
    z, phi = sk.ring_pix2ang(nside, np.arange(12 * nside * nside))
    m = sph_harm_y(ell, 0, np.arccos(z), phi).real
    cl = sk.angular_power(m, nside, 10)
    assert abs(cl[ell] * (2 * ell + 1) - 1.0) < 1e-2
    others = np.delete(cl, ell)
    assert others.max() < 1e-4 * cl[ell]


def test_compare_maps_without_records_reports_none():
    import warnings
    nside = 4
    full = np.ones(12 * nside * nside)
    empty = np.zeros_like(full)
    with warnings.catch_warnings():
        warnings.simplefilter("error")   # no divide-by-zero warnings either
        for a, b, names in ((empty, empty, ["a", "b"]), (full, empty, ["b"]),
                            (empty, full, ["a"])):
            r = sk.compare_maps(a, b, nside, 4)
            assert r["no_records"] == names
            assert r["max_abs_pixel_difference_over_mean"] is None
            assert r["max_abs_Cl_ratio_minus_1"] is None
    r = sk.compare_maps(full, full, nside, 4)
    assert "no_records" not in r and r["max_abs_pixel_difference_over_mean"] == 0.0

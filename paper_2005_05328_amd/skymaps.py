"""Sky-projected lightcone maps and their angular power (accuracy diagnostics of the lightcone
output, paper Sec. 3.1.3 and the sky-map comparison of Sec. 3.2).

Equal-area pixels: the HEALPix ring scheme (Gorski et al. 2005, ApJ 622, 759): 12 nside^2
pixels on 4 nside - 1 iso-latitude rings; the polar caps (|z| > 2/3) and the equatorial belt
use the published ang2pix / pix2ang relations, restated here.  Angular power: a_lm summed
over pixel centres with equal weights 4 pi / N_pix, C_l = sum_m |a_lm|^2 / (2 l + 1).

Host-side diagnostics only (numpy, torch for the record arrays already on the device); no
part of the gravity step.
"""
from __future__ import annotations

import math

import numpy as np


def ring_ang2pix(nside: int, z, phi):
    """Ring-scheme pixel of directions with cos(theta) = z and azimuth phi in [0, 2 pi).
    Works on torch tensors or numpy arrays (same module for z and phi)."""
    xp = _xp(z)
    n = nside
    za = xp.abs(z)
    tt = xp.remainder(phi, 2.0 * math.pi) / (0.5 * math.pi)   # in [0, 4)
    # equatorial belt
    t1 = n * (0.5 + tt)
    t2 = n * z * 0.75
    jp = xp.floor(t1 - t2)
    jm = xp.floor(t1 + t2)
    ir = n + 1 + jp - jm                                        # 1 .. 2n + 1
    kshift = 1 - _mod(ir, 2, xp)
    ip = xp.floor((jp + jm - n + kshift + 1) / 2)
    ip = _mod(ip, 4 * n, xp)
    pix_eq = 2 * n * (n - 1) + (ir - 1) * 4 * n + ip
    # polar caps
    tp = tt - xp.floor(tt)
    tmp = n * xp.sqrt(xp.clip(3.0 * (1.0 - za), 0.0, None))
    jp2 = xp.floor(tp * tmp)
    jm2 = xp.floor((1.0 - tp) * tmp)
    ir2 = jp2 + jm2 + 1                                         # ring from the nearer pole
    ip2 = _mod(xp.floor(tt * ir2), 4 * ir2, xp)
    pix_n = 2 * ir2 * (ir2 - 1) + ip2
    pix_s = 12 * n * n - 2 * ir2 * (ir2 + 1) + ip2
    pix_cap = xp.where(z > 0, pix_n, pix_s)
    pix = xp.where(za <= 2.0 / 3.0, pix_eq, pix_cap)
    return pix.long() if hasattr(pix, "long") else pix.astype(np.int64)


def ring_pix2ang(nside: int, pix: np.ndarray):
    """Centres (z = cos theta, phi) of ring-scheme pixels (numpy)."""
    n = nside
    pix = np.asarray(pix, np.int64)
    npix = 12 * n * n
    ncap = 2 * n * (n - 1)
    z = np.empty(pix.shape, np.float64)
    phi = np.empty(pix.shape, np.float64)
    north = pix < ncap
    south = pix >= npix - ncap
    belt = ~north & ~south
    p = pix[north]
    iring = np.floor((1 + np.sqrt(1 + 2 * p)) / 2).astype(np.int64)
    iphi = p + 1 - 2 * iring * (iring - 1)
    z[north] = 1.0 - iring ** 2 / (3.0 * n * n)
    phi[north] = (iphi - 0.5) * math.pi / (2.0 * iring)
    p = pix[belt] - ncap
    iring = p // (4 * n) + n
    iphi = p % (4 * n) + 1
    fodd = 0.5 * (1 + (iring + n) % 2)
    z[belt] = (2 * n - iring) * 2.0 / (3.0 * n)
    phi[belt] = (iphi - fodd) * math.pi / (2.0 * n)
    p = npix - pix[south]
    iring = np.floor((1 + np.sqrt(2 * p - 1)) / 2).astype(np.int64)
    iphi = 4 * iring + 1 - (p - 2 * iring * (iring - 1))
    z[south] = -1.0 + iring ** 2 / (3.0 * n * n)
    phi[south] = (iphi - 0.5) * math.pi / (2.0 * iring)
    return z, phi


def sky_map(d, weights, nside: int, out=None):
    """Weighted counts of offsets d (n x 3, observer at the origin) per ring pixel; added to
    `out` (length 12 nside^2) when given.  Torch tensors in, torch tensor out."""
    import torch
    r = torch.sqrt((d * d).sum(1))
    ok = r > 0
    z = torch.where(ok, d[:, 2] / torch.where(ok, r, torch.ones_like(r)), torch.zeros_like(r))
    z = torch.clamp(z, -1.0, 1.0)
    phi = torch.remainder(torch.atan2(d[:, 1], d[:, 0]), 2.0 * math.pi)
    pix = ring_ang2pix(nside, z, phi)
    npix = 12 * nside * nside
    if out is None:
        out = torch.zeros(npix, dtype=torch.float64, device=d.device)
    out.index_add_(0, pix, weights.to(torch.float64))
    return out


def angular_power(m: np.ndarray, nside: int, lmax: int) -> np.ndarray:
    """C_l, l = 0..lmax, of a ring-ordered map (pixel-centre quadrature).  Pixels of a ring
    share their colatitude, so Y_lm(theta, phi) = Y_lm(theta, 0) e^(i m phi) splits into a
    per-ring sum over azimuths and a sum over rings."""
    from scipy.special import sph_harm_y
    m = np.asarray(m, np.float64)
    npix = 12 * nside * nside
    z, phi = ring_pix2ang(nside, np.arange(npix))
    zr, ring = np.unique(np.round(z, 12), return_inverse=True)
    theta_r = np.arccos(np.clip(zr, -1.0, 1.0))
    w = 4.0 * math.pi / npix
    cl = np.zeros(lmax + 1)
    for mm in range(lmax + 1):
        f = (np.bincount(ring, weights=m * np.cos(mm * phi), minlength=zr.size)
             - 1j * np.bincount(ring, weights=m * np.sin(mm * phi), minlength=zr.size))
        for ell in range(mm, lmax + 1):
            y = sph_harm_y(ell, mm, theta_r, 0.0).real
            a = w * np.sum(y * f)
            cl[ell] += abs(a) ** 2 * (1.0 if mm == 0 else 2.0)
    return cl / (2 * np.arange(lmax + 1) + 1)


def compare_maps(map_a, map_b, nside: int, lmax: int) -> dict:
    """Pixel and angular-power agreement of two sky maps (b the reference).  When either map
    holds no mass (no lightcone records) nothing can be compared: every figure is None and
    `no_records` names the empty map(s)."""
    a = np.asarray(map_a, np.float64)
    b = np.asarray(map_b, np.float64)
    empty = [name for name, m in (("a", a), ("b", b)) if not m.sum() > 0.0]
    if empty:
        return {"nside": nside, "lmax": lmax, "no_records": empty,
                "max_abs_pixel_difference_over_mean": None,
                "rms_pixel_difference_over_mean": None, "max_abs_Cl_ratio_minus_1": None}
    mean = b.mean()
    ca = angular_power(a / a.mean() - 1.0, nside, lmax)
    cb = angular_power(b / mean - 1.0, nside, lmax)
    # multipoles where the reference has power (a uniform reference has none: then the two
    # agree only if neither has any)
    has = cb[1:] > 0.0
    if has.any():
        cl_dev = float(np.abs(ca[1:][has] / cb[1:][has] - 1.0).max())
    else:
        cl_dev = 0.0 if not (ca[1:] > 0.0).any() else None
    return {"nside": nside, "lmax": lmax,
            "max_abs_pixel_difference_over_mean": float(np.abs(a - b).max() / mean),
            "rms_pixel_difference_over_mean": float(np.sqrt(np.mean((a - b) ** 2)) / mean),
            "max_abs_Cl_ratio_minus_1": cl_dev}


def _xp(a):
    try:
        import torch
        if isinstance(a, torch.Tensor):
            return torch
    except ImportError:
        pass
    return np


def _mod(a, b, xp):
    return a - b * xp.floor(a / b)

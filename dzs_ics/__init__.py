"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the benchmark.

This module only *generates inputs*: particle lattices, Gaussian random fields with
Zel'dovich displacements, uniform and clustered random point sets, and merged-particle
(mixed multiplicity) states.  It holds none of the gravity step's arithmetic; it is
imported by both sides of every parity check, and by nothing on the product's compute path.

Randomness comes from numpy's Philox-4x32-10 counter-based generator (Salmon et al.
2011), seeded explicitly, so every input is reproducible from its seed.

Units follow the usual cosmological N-body convention: lengths in Mpc/h, velocities in
km/s, masses in 1e10 Msun/h.  Momenta are p = a^2 dx/dt (comoving).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

G_CODE = 43.0091          # gravitational constant, (Mpc/h) (km/s)^2 / (1e10 Msun/h)
H0 = 100.0                # km/s / (Mpc/h)
C_LIGHT = 299792.458      # km/s

__all__ = [
    "ParticleSet", "rng", "lattice", "uniform_random", "clustered_random",
    "zeldovich", "mean_matter_density", "particle_mass", "power_bbks", "power_powerlaw",
    "merged_state", "growth_factor", "growth_rate", "hubble",
]


def rng(seed: int) -> np.random.Generator:
    """A numpy Generator on the Philox-4x32-10 counter-based bit generator."""
    return np.random.Generator(np.random.Philox(int(seed)))


@dataclass
class ParticleSet:
    """Structure-of-arrays particle state (host, numpy)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    px: np.ndarray
    py: np.ndarray
    pz: np.ndarray
    mult: np.ndarray   # uint32 multiplicity: mass = mult * m0
    id: np.ndarray     # uint32 particle id
    type: np.ndarray   # uint8: 0 original, 1 merged
    L: float

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def copy(self) -> "ParticleSet":
        return ParticleSet(*(a.copy() for a in (self.x, self.y, self.z, self.px, self.py,
                                                 self.pz, self.mult, self.id, self.type)), L=self.L)

    def take(self, idx) -> "ParticleSet":
        return ParticleSet(*(a[idx].copy() for a in (self.x, self.y, self.z, self.px, self.py,
                                                      self.pz, self.mult, self.id, self.type)), L=self.L)


def _wrap(v: np.ndarray, L: float) -> np.ndarray:
    v = np.mod(v, L)
    v[v >= L] = 0.0
    return v


def _make(x, y, z, px, py, pz, L, mult=None, ids=None, typ=None) -> ParticleSet:
    n = x.shape[0]
    return ParticleSet(
        np.ascontiguousarray(x, np.float64), np.ascontiguousarray(y, np.float64),
        np.ascontiguousarray(z, np.float64), np.ascontiguousarray(px, np.float64),
        np.ascontiguousarray(py, np.float64), np.ascontiguousarray(pz, np.float64),
        np.ones(n, np.uint32) if mult is None else np.ascontiguousarray(mult, np.uint32),
        np.arange(n, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, np.uint32),
        np.zeros(n, np.uint8) if typ is None else np.ascontiguousarray(typ, np.uint8),
        float(L))


def lattice(n_side: int, L: float) -> ParticleSet:
    """Cubic lattice q = (i + 1/2) * lambda, lambda = L / n_side, at rest."""
    lam = L / n_side
    i = (np.arange(n_side, dtype=np.float64) + 0.5) * lam
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    zero = np.zeros(n_side ** 3)
    return _make(X.ravel(), Y.ravel(), Z.ravel(), zero, zero.copy(), zero.copy(), L)


def uniform_random(n: int, L: float, seed: int, vel: float = 0.0) -> ParticleSet:
    """n points uniform in [0,L)^3 with Gaussian momenta of rms `vel` per component."""
    g = rng(seed)
    pos = g.random((3, n)) * L
    mom = g.standard_normal((3, n)) * vel
    return _make(_wrap(pos[0], L), _wrap(pos[1], L), _wrap(pos[2], L), mom[0], mom[1], mom[2], L)


def clustered_random(n: int, L: float, seed: int, n_clumps: int = 8, frac: float = 0.7,
                     r_clump: float | None = None, vel: float = 300.0) -> ParticleSet:
    """A clustered point set: `frac` of the points in Plummer-like clumps, the rest uniform.

    Used to give trees realistic depth and occupancy spread (dense halos plus voids).
    """
    g = rng(seed)
    r_clump = L / 40.0 if r_clump is None else r_clump
    n_cl = int(n * frac)
    centres = g.random((n_clumps, 3)) * L
    which = g.integers(0, n_clumps, n_cl)
    # Plummer radial profile: r = a / sqrt(u^(-2/3) - 1)
    u = np.clip(g.random(n_cl), 1e-6, 0.999)
    r = r_clump / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    r = np.minimum(r, 10 * r_clump)
    d = g.standard_normal((n_cl, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pos_cl = centres[which] + d * r[:, None]
    pos_un = g.random((n - n_cl, 3)) * L
    pos = np.concatenate([pos_cl, pos_un], axis=0)
    perm = g.permutation(n)
    pos = pos[perm]
    mom = g.standard_normal((n, 3)) * vel
    return _make(_wrap(pos[:, 0].copy(), L), _wrap(pos[:, 1].copy(), L), _wrap(pos[:, 2].copy(), L),
                 mom[:, 0], mom[:, 1], mom[:, 2], L)


def merged_state(ps: ParticleSet, seed: int, frac: float = 0.3, max_mult: int = 64) -> ParticleSet:
    """Give a random subset of particles a multiplicity > 1 and type 1 (a mixed-mass set)."""
    g = rng(seed)
    out = ps.copy()
    sel = g.random(ps.n) < frac
    out.mult[sel] = g.integers(2, max_mult + 1, int(sel.sum())).astype(np.uint32)
    out.type[sel] = 1
    return out


# ----------------------------------------------------------------------------------------
# Initial-condition cosmology: flat LCDM, used only to set the amplitude and the velocity of
# the linear-theory Zel'dovich start.
# ----------------------------------------------------------------------------------------

def hubble(a, om=0.3):
    """H(a) in km/s/(Mpc/h) for flat LCDM without radiation."""
    return H0 * np.sqrt(om * np.asarray(a, dtype=np.float64) ** -3 + (1.0 - om))


def _growth_integral(a, om=0.3, n=4000):
    # Heath (1977): D(a) proportional to H(a) * int_0^a da' / (a' H(a'))^3.  The integrand
    # tends to a'^{3/2}/(H0^3 om^{3/2}) as a' -> 0, so a midpoint rule in s = a'^{5/2} is smooth.
    s_max = a ** 2.5
    s = (np.arange(n) + 0.5) / n * s_max
    ap = s ** 0.4
    da_ds = 0.4 * s ** (-0.6)
    f = 1.0 / (ap * hubble(ap, om)) ** 3 * da_ds
    return f.sum() * s_max / n


def growth_factor(a, om=0.3):
    """Linear growth D(a), normalised to D(1) = 1."""
    d = hubble(a, om) * _growth_integral(a, om)
    return d / (hubble(1.0, om) * _growth_integral(1.0, om))


def growth_rate(a, om=0.3):
    """f = dlnD/dlna from the Heath form D = H I: f = dlnH/dlna + a / ((aH)^3 I)."""
    e2 = om * a ** -3 + (1.0 - om)
    dlnh = -1.5 * om * a ** -3 / e2
    return dlnh + a / ((a * hubble(a, om)) ** 3 * _growth_integral(a, om))


def mean_matter_density(om=0.3):
    """Comoving mean matter density, (1e10 Msun/h) / (Mpc/h)^3."""
    return om * 3.0 * H0 ** 2 / (8.0 * math.pi * G_CODE)


def particle_mass(L: float, n_init: int, om=0.3) -> float:
    """m0 = rho_bar L^3 / N_init: the mass of a multiplicity-1 particle."""
    return mean_matter_density(om) * L ** 3 / n_init


def power_powerlaw(k, index=-2.0):
    k = np.asarray(k, dtype=np.float64)
    return np.where(k > 0, np.abs(np.where(k > 0, k, 1.0)) ** index, 0.0)


def power_bbks(k, gamma=0.21, ns=0.96):
    """BBKS (1986) transfer-function shape times k^ns (unnormalised)."""
    k = np.asarray(k, dtype=np.float64)
    q = np.where(k > 0, k / gamma, 1.0)
    t = np.log(1 + 2.34 * q) / (2.34 * q) * (1 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3
                                              + (6.71 * q) ** 4) ** -0.25
    return np.where(k > 0, k ** ns * t ** 2, 0.0)


def _sigma_r(pk, r=8.0):
    # sigma^2(R) = 1/(2 pi^2) int k^2 P(k) W^2(kR) dk, top-hat window, log-spaced midpoint rule
    lnk = np.linspace(np.log(1e-5), np.log(1e3), 200001)
    k = np.exp(lnk)
    x = k * r
    w = 3 * (np.sin(x) - x * np.cos(x)) / x ** 3
    integrand = k ** 3 * pk(k) * w ** 2
    return math.sqrt(np.trapezoid(integrand, lnk) / (2 * math.pi ** 2))


def zeldovich(n_side: int, L: float, a_init: float, seed: int, spectrum: str = "bbks",
              sigma8: float = 0.8, om: float = 0.3) -> ParticleSet:
    """Lattice + Zel'dovich displacement from a seeded Gaussian random field.

    The white-noise field is drawn in real space on the n_side^3 grid (Philox), so the
    Fourier modes are Hermitian by construction; the Nyquist planes and k = 0 are zeroed.
    Displacement psi_k = i k delta_k / k^2 (so delta = -div psi), scaled by D(a)/D(1);
    momentum p = a^2 H f psi.  Positions are wrapped into [0, L).  One displacement component
    is held at a time (a 1024^3 lattice needs ~80 GB of host memory); FFTs use every core.
    """
    import os
    import scipy.fft as sfft
    workers = os.cpu_count() or 1
    pk = {"bbks": power_bbks, "powerlaw": power_powerlaw}[spectrum]
    amp = (sigma8 / _sigma_r(pk)) ** 2
    g = rng(seed)
    dk = sfft.rfftn(g.standard_normal((n_side, n_side, n_side)), workers=workers)
    kf = 2 * np.pi / L
    k1 = np.fft.fftfreq(n_side, 1.0 / n_side) * kf
    k3 = np.fft.rfftfreq(n_side, 1.0 / n_side) * kf
    k2 = (k1 ** 2)[:, None, None] + (k1 ** 2)[None, :, None] + (k3 ** 2)[None, None, :]
    cell_vol = (L / n_side) ** 3
    dk *= np.sqrt(amp * pk(np.sqrt(k2)) / cell_vol)
    nyq = n_side // 2
    if n_side % 2 == 0:
        dk[nyq, :, :] = 0
        dk[:, nyq, :] = 0
        dk[:, :, nyq] = 0
    dk[0, 0, 0] = 0
    k2[0, 0, 0] = 1.0
    dk /= k2
    del k2
    dfac = growth_factor(a_init, om)
    vfac = a_init ** 2 * hubble(a_init, om) * growth_rate(a_init, om)
    q = (np.arange(n_side, dtype=np.float64) + 0.5) * (L / n_side)
    shape = (n_side, n_side, n_side)
    pos, mom = [], []
    max_disp = 0.0
    for axis, kd in enumerate((k1[:, None, None], k1[None, :, None], k3[None, None, :])):
        psi = sfft.irfftn(1j * kd * dk, s=shape, axes=(0, 1, 2), workers=workers).ravel()
        psi *= dfac
        max_disp = max(max_disp, float(np.abs(psi).max()))
        base = np.broadcast_to(q.reshape([-1 if d == axis else 1 for d in range(3)]), shape)
        pos.append(_wrap(base.ravel() + psi, L))
        mom.append(vfac * psi)
        del psi
    del dk
    ps = _make(pos[0], pos[1], pos[2], mom[0], mom[1], mom[2], L)
    ps.max_disp = max_disp  # type: ignore[attr-defined]
    return ps

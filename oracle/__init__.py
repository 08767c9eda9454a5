"""FP64 CPU oracle for the DZS gravity step — TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import this package.  It shares no code with the GPU library (``paper_2005_05328_amd``):
its heavy loops live in ``dzs_oracle.c`` (plain C, compiled with gcc), the rest is numpy and
scipy written to be read against the paper (Garaldi, Nori & Baldi 2020, arXiv:2005.05328).

What each part follows:
  * Morton keys / tree cubes ........ Sec. 2.1 (oct-tree: root = box, octants recursively)
  * DZS coarsening ................... Sec. 2.2, 2.2.1, eqs. (1) and (3), l_max cap
  * short-range force ................ Sec. 2.1 TreePM split, by direct summation
  * PM long-range force .............. Sec. 2.1 (grid density, Poisson solve in Fourier space,
                                       exponential split kernel)
  * softening rescale ................ Sec. 2.2, eps ∝ (M/M_init)^(1/3)
  * lightcone crossing ............... Sec. 1 footnote (R_lc) and Sec. 3.1.3 (on-the-fly
                                       shell output), in its zero-width every-step limit
  * kick-drift-kick, cosmology ....... not specified by the paper (readings listed in the
                                       design notes): flat LCDM, p = a^2 dx/dt, KDK in a.
  * individual time steps ............ Sec. 2.1 (power-of-two steps), Sec. 2.2 (DZS at
                                       global steps, the out-of-lightcone limiter); the
                                       long-range force on the global step only (the TreePM
                                       split carried into time)

Parity status: every function here is pinned by the ``-m "not gpu"`` tests against closed
forms, invariants or brute force, except the tree-walk force at a non-zero opening angle
(an approximation with no closed form: parity unpinned beyond the direct sum itself).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dzs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_dzs_oracle.so")

# Code units: Mpc/h, km/s, 1e10 Msun/h.
G = 43.0091
H0 = 100.0
C_LIGHT = 299792.458
OMEGA_M = 0.3
OMEGA_L = 0.7


def build(force: bool = True) -> str:
    """Compile the oracle's C part with gcc (IEEE FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        d, i64, u32p, u8p, dp, i64p, u64p = (ctypes.c_double, ctypes.c_int64,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p)
        L.orc_morton_keys.argtypes = [i64, dp, dp, dp, d, u64p]
        L.orc_coarsen.argtypes = [i64, dp, dp, dp, dp, dp, dp, u32p, u32p, u8p, d, dp, d, d, d,
                                  ctypes.c_int, ctypes.c_int, d, d, dp, dp, dp, dp,
                                  dp, dp, dp, dp, dp, dp, u32p, u32p, u8p, i64p, i64p]
        L.orc_coarsen.restype = i64
        L.orc_a_min.argtypes = [i64, dp, dp, dp, dp, dp, dp, d, dp, d]
        L.orc_a_min.restype = d
        L.orc_merge_thresholds.argtypes = [d, d, d, d, dp]
        L.orc_short_range.argtypes = [i64, dp, dp, dp, u32p, d, d, d, d, d, d, i64, i64p, dp, dp, dp]
        L.orc_cic_deposit.argtypes = [i64, dp, dp, dp, u32p, d, ctypes.c_int, d, dp]
        L.orc_cic_interp.argtypes = [i64, dp, dp, dp, d, ctypes.c_int, dp, dp]
        L.orc_g_soft.argtypes = [d, d]
        L.orc_g_soft.restype = d
        L.orc_split_S.argtypes = [d]
        L.orc_split_S.restype = d
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Box:
    """Periodic box: side L, multiplicity-1 particle mass m0, softening eps0, G."""
    L: float
    m0: float
    eps0: float
    G: float = G


# ======================================================================================
# Morton keys (tree cubes)
# ======================================================================================

def morton_keys(x, y, z, L) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = np.empty(x.shape[0], np.uint64)
    lib().orc_morton_keys(x.shape[0], _p(x), _p(y), _p(z), float(L), _p(out))
    return out


# ======================================================================================
# DZS coarsening (Sec. 2.2, eqs. 1 and 3)
# ======================================================================================

def merge_thresholds(L, R_lc, b, theta) -> np.ndarray:
    out = np.empty(22, np.float64)
    lib().orc_merge_thresholds(float(L), float(R_lc), float(b), float(theta), _p(out))
    return out


def k_min_for(n_side: int, lmax_over_lambda: int) -> int:
    """Shallowest level allowed to merge: l_k = L/2^k <= l_max = j*lambda, integers only.

    l_k <= j L / n_side  <=>  n_side <= j 2^k; the smallest such k.
    """
    k = 0
    while n_side > lmax_over_lambda * (1 << k):
        k += 1
    return k


def coarsen(ps, x_obs, R_lc, b, theta, k_min, alpha_dyn=None, g=None, Gm0=None):
    """Top-down merge walk.  Returns (new particle dict, group_of[old] -> new, n_merged_nodes).

    Geometric criterion (eq. 1 with eq. 3) by default; with `alpha_dyn` the dynamical one
    (eq. 2 with eq. 3 and the in-lightcone minimum of the previous accelerations `g`, shape
    (3, n), Sec. 2.2.1), which also needs Gm0 = G m0.  `theta` is ignored then."""
    n = ps.n
    outs = {k: np.empty(n, np.float64) for k in ("x", "y", "z", "px", "py", "pz")}
    omult = np.empty(n, np.uint32)
    oid = np.empty(n, np.uint32)
    otype = np.empty(n, np.uint8)
    group_of = np.empty(n, np.int64)
    nm = np.zeros(1, np.int64)
    xo = _f64(x_obs)
    arrs = [_f64(ps.x), _f64(ps.y), _f64(ps.z), _f64(ps.px), _f64(ps.py), _f64(ps.pz)]
    mult = np.ascontiguousarray(ps.mult, np.uint32)
    ids = np.ascontiguousarray(ps.id, np.uint32)
    typ = np.ascontiguousarray(ps.type, np.uint8)
    amin = np.zeros(1, np.float64)
    if alpha_dyn is None:
        crit, alpha, gm0, gp = 0, 0.0, 0.0, [None, None, None]
        theta = float(theta)
    else:
        if g is None or Gm0 is None:
            raise ValueError("the dynamical criterion needs g and Gm0")
        crit, alpha, gm0 = 1, float(alpha_dyn), float(Gm0)
        gg = [_f64(g[0]), _f64(g[1]), _f64(g[2])]
        gp = [_p(a) for a in gg]
        theta = 1.0 if theta is None else float(theta)
    n_out = lib().orc_coarsen(n, *[_p(a) for a in arrs], _p(mult), _p(ids), _p(typ), float(ps.L),
                              _p(xo), float(R_lc), float(b), theta, int(k_min),
                              crit, alpha, gm0, *gp, _p(amin),
                              *[_p(outs[k]) for k in ("x", "y", "z", "px", "py", "pz")],
                              _p(omult), _p(oid), _p(otype), _p(group_of), _p(nm))
    res = {k: v[:n_out].copy() for k, v in outs.items()}
    res["mult"] = omult[:n_out].copy()
    res["id"] = oid[:n_out].copy()
    res["type"] = otype[:n_out].copy()
    res["a_min"] = float(amin[0])
    return res, group_of, int(nm[0])


def a_min_lightcone(x, y, z, g, L, x_obs, R_lc, b) -> float:
    """Smallest |g| among particles within R_lc + b of the observer (min image); +inf if none."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    gg = [_f64(g[0]), _f64(g[1]), _f64(g[2])]
    return lib().orc_a_min(x.shape[0], _p(x), _p(y), _p(z), *[_p(a) for a in gg], float(L),
                           _p(_f64(x_obs)), float(R_lc) + float(b))


# ======================================================================================
# Short-range force by direct summation (Sec. 2.1)
# ======================================================================================

def g_soft(r, h) -> float:
    return lib().orc_g_soft(float(r), float(h))


def split_S(u) -> float:
    return lib().orc_split_S(float(u))


def short_range(x, y, z, mult, box: Box, r_s, r_cut, targets=None):
    x, y, z = _f64(x), _f64(y), _f64(z)
    mult = np.ascontiguousarray(mult, np.uint32)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        targets = np.ascontiguousarray(targets, np.int64)
        nt, tp = targets.shape[0], _p(targets)
    g = [np.empty(nt, np.float64) for _ in range(3)]
    lib().orc_short_range(n, _p(x), _p(y), _p(z), _p(mult), box.L, box.m0, box.eps0, box.G,
                          float(r_s), float(r_cut), nt, tp, _p(g[0]), _p(g[1]), _p(g[2]))
    return np.stack(g)


# ======================================================================================
# PM long-range force (Sec. 2.1): CIC density -> FFT -> Gaussian-filtered Green's function
# -> inverse FFT -> 4-point finite-difference gradient -> CIC interpolation.
# ======================================================================================

def cic_deposit(x, y, z, mult, L, ng, m0) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    mult = np.ascontiguousarray(mult, np.uint32)
    rho = np.empty((ng, ng, ng), np.float64)
    lib().orc_cic_deposit(x.shape[0], _p(x), _p(y), _p(z), _p(mult), float(L), int(ng),
                          float(m0), _p(rho))
    return rho


def cic_interp(x, y, z, L, mesh) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    mesh = np.ascontiguousarray(mesh, np.float64)
    out = np.empty(x.shape[0], np.float64)
    lib().orc_cic_interp(x.shape[0], _p(x), _p(y), _p(z), float(L), int(mesh.shape[0]),
                         _p(mesh), _p(out))
    return out


def green_kernel(L, ng, r_s, Gc=G):
    """Multiplier on rho_k giving psi_k: -4 pi G exp(-k^2 r_s^2) / (k^2 W(k)^2), psi_0 = 0.

    W(k) = prod_d sinc^2(k_d Delta / 2) is the CIC assignment window; dividing by W^2
    undoes it once for the deposit and once for the interpolation.
    """
    delta = L / ng
    n1 = np.fft.fftfreq(ng, 1.0 / ng)
    n3 = np.fft.rfftfreq(ng, 1.0 / ng)
    k1 = 2 * np.pi * n1 / L
    k3 = 2 * np.pi * n3 / L

    def sinc2(k):
        h = 0.5 * k * delta
        s = np.ones_like(h)
        nz = h != 0
        s[nz] = np.sin(h[nz]) / h[nz]
        return s * s

    KX, KY, KZ = np.meshgrid(k1, k1, k3, indexing="ij")
    WX, WY, WZ = np.meshgrid(sinc2(k1), sinc2(k1), sinc2(k3), indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    W = WX * WY * WZ
    k2s = np.where(k2 > 0, k2, 1.0)
    gk = -4 * np.pi * Gc * np.exp(-k2 * r_s * r_s) / (k2s * W * W)
    gk[0, 0, 0] = 0.0
    return gk


def pm_potential(rho, L, r_s, Gc=G):
    ng = rho.shape[0]
    rk = np.fft.rfftn(rho)
    return np.fft.irfftn(rk * green_kernel(L, ng, r_s, Gc), s=rho.shape, axes=(0, 1, 2))


def fd4_gradient(psi, L):
    """g = -grad psi with the 4-point central difference:
    g_j = -(1/Delta) [ 2/3 (psi_{j+1} - psi_{j-1}) - 1/12 (psi_{j+2} - psi_{j-2}) ]."""
    delta = L / psi.shape[0]
    out = []
    for ax in range(3):
        p1 = np.roll(psi, -1, axis=ax)
        m1 = np.roll(psi, 1, axis=ax)
        p2 = np.roll(psi, -2, axis=ax)
        m2 = np.roll(psi, 2, axis=ax)
        out.append(-(2.0 / 3.0 * (p1 - m1) - 1.0 / 12.0 * (p2 - m2)) / delta)
    return out


def pm_force(x, y, z, mult, box: Box, ng, r_s):
    rho = cic_deposit(x, y, z, mult, box.L, ng, box.m0)
    psi = pm_potential(rho, box.L, r_s, box.G)
    return np.stack([cic_interp(x, y, z, box.L, gm) for gm in fd4_gradient(psi, box.L)])


def total_force(x, y, z, mult, box: Box, ng, r_s, r_cut):
    return pm_force(x, y, z, mult, box, ng, r_s) + short_range(x, y, z, mult, box, r_s, r_cut)


# ======================================================================================
# Cosmology (flat LCDM, no radiation): the kick / drift integrals and the comoving distance
# ======================================================================================

def E(a, om=OMEGA_M):
    """H(a)/H0 for flat LCDM without radiation."""
    return math.sqrt(om / a ** 3 + (1.0 - om))


def _quad(f, a, b):
    from scipy.integrate import quad
    val, _ = quad(f, a, b, epsabs=0.0, epsrel=1.2e-14, limit=400)
    return val


def kick_factor(a0, a1, om=OMEGA_M):
    """K(a0,a1) = int da / (a^2 H(a)): dp = g K for p = a^2 dx/dt, dp/dt = g/a."""
    return _quad(lambda a: 1.0 / (a * a * H0 * E(a, om)), a0, a1)


def drift_factor(a0, a1, om=OMEGA_M):
    """D(a0,a1) = int da / (a^3 H(a)): dx = p D."""
    return _quad(lambda a: 1.0 / (a ** 3 * H0 * E(a, om)), a0, a1)


def chi(a, om=OMEGA_M):
    """Comoving distance to scale factor a, Mpc/h: (c/H0) int_a^1 da / (a^2 E(a))."""
    return C_LIGHT * _quad(lambda x: 1.0 / (x * x * H0 * E(x, om)), a, 1.0)


def chi_inverse(d):
    from scipy.optimize import brentq
    if d <= 0:
        return 1.0
    return brentq(lambda a: chi(a) - d, 1e-4, 1.0, xtol=1e-16, rtol=8.9e-16, maxiter=200)


# ======================================================================================
# Kick, drift and lightcone crossing
# ======================================================================================

def kick(p, g, K):
    """p <- p + g K (one product, one sum)."""
    return p + g * K


def wrap(x, L):
    """x - L floor(x/L); a result equal to L becomes 0."""
    w = x - L * np.floor(x / L)
    w[w >= L] = 0.0
    return w


def drift(x, p, D, L):
    """Unwrapped drifted coordinate x + p D, then wrapped into [0, L)."""
    return wrap(x + p * D, L)


def min_image(d, L):
    d = np.array(d, dtype=np.float64, copy=True)
    hi = d >= 0.5 * L
    lo = d < -0.5 * L
    d[hi] -= L
    d[lo] += L
    return d


def lightcone_select(x, y, z, px, py, pz, L, x_obs, D, chi2_0, chi2_1):
    """Crossing test over one drift a_n -> a_{n+1}.

    The lightcone sphere (radius chi(a), the comoving distance the light reaching the observer
    at a = 1 left from at a) shrinks as a grows.  With d0 the minimum-image offset from the
    observer at a_n, and d1 the minimum-image offset of the drifted, wrapped position at
    a_{n+1} (exactly the next drift's d0), a particle is on the past lightcone when
    f = |d|^2 - chi^2 changes sign from negative to non-negative: emit iff f0 < 0 <= f1.
    Because f1 of one drift is f0 of the next, each particle is emitted once.
    Returns (mask, d0 (3,n), f0, f1).
    """
    d0 = np.stack([min_image(_f64(c) - xo, L) for c, xo in zip((x, y, z), x_obs)])
    pp = np.stack([_f64(px), _f64(py), _f64(pz)])
    d1 = np.stack([min_image(drift(_f64(c), pc, D, L) - xo, L)
                   for c, pc, xo in zip((x, y, z), pp, x_obs)])
    f0 = (d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2]) - chi2_0
    f1 = (d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]) - chi2_1
    mask = (f0 < 0) & (f1 >= 0)
    return mask, d0, f0, f1


def crossing_time(d0, p, a0, a1):
    """Solve |d0 + p D(a0,a)| = chi(a) for a in [a0, a1] with Brent's method on quadrature."""
    from scipy.optimize import brentq
    d0 = np.asarray(d0, np.float64)
    p = np.asarray(p, np.float64)

    def F(a):
        d = d0 + p * drift_factor(a0, a)
        return float(d @ d) - chi(a) ** 2

    fa, fb = F(a0), F(a1)
    if fa >= 0:
        return a0
    if fb <= 0:
        return a1
    return brentq(F, a0, a1, xtol=1e-15, rtol=8.9e-16, maxiter=200)


def lightcone_records(ps, x_obs, a0, a1, D, chi2_0, chi2_1, solve=True, limit=None):
    """Records {id, mult, a_cross, d(a_cross)[3], p[3]} for the particles selected above."""
    mask, d0, _, _ = lightcone_select(ps.x, ps.y, ps.z, ps.px, ps.py, ps.pz, ps.L, x_obs, D,
                                      chi2_0, chi2_1)
    idx = np.nonzero(mask)[0]
    if limit is not None:
        idx = idx[:limit]
    rec = {"index": idx, "id": ps.id[idx].copy(), "mult": ps.mult[idx].copy()}
    if solve:
        ac = np.empty(idx.shape[0])
        dc = np.empty((idx.shape[0], 3))
        for r, i in enumerate(idx):
            p = np.array([ps.px[i], ps.py[i], ps.pz[i]])
            ac[r] = crossing_time(d0[:, i], p, a0, a1)
            dc[r] = d0[:, i] + p * drift_factor(a0, ac[r])
        rec["a_cross"] = ac
        rec["d"] = dc
        rec["p"] = np.stack([ps.px[idx], ps.py[idx], ps.pz[idx]], axis=1)
    return rec


def step_factors(a0, a1):
    """K(a0, a_h), D(a0, a1), K(a_h, a1) with a_h = sqrt(a0 a1), and chi^2 at both ends."""
    ah = math.sqrt(a0 * a1)
    c0, c1 = chi(a0), chi(a1)
    return {"K1": kick_factor(a0, ah), "D": drift_factor(a0, a1), "K2": kick_factor(ah, a1),
            "chi2_0": c0 * c0, "chi2_1": c1 * c1, "R_lc1": c1}


def kdk_step(ps, g, box: Box, fac, ng, r_s, r_cut, x_obs, coarsen_params=None, solve=True,
             lc_limit=None):
    """One kick-drift-kick step a_n -> a_{n+1} on a copy of `ps` (a dzs_ics.ParticleSet).

    Order (coarsening placed as the paper places DZS: at a global step, before the tree
    rebuild and the force, so the merged particles get fresh accelerations, Sec. 2.2):
      1. p += g K(a_n, a_h)
      2. lightcone crossings over the drift, on the pre-drift positions and the kicked p
      3. x = wrap(x + p D(a_n, a_{n+1}))
      4. optional DZS coarsening at a_{n+1} (positions at a_{n+1}, momenta at a_h)
      5. g = PM + short-range force of the (new) set
      6. p += g K(a_h, a_{n+1})
    `fac` holds K1, D, K2, chi2_0, chi2_1 (see step_factors) and a0, a1.
    Returns (new state, new g (3,n), lightcone records, coarsening result or None).
    """
    s = ps.copy()
    s.px = kick(s.px, g[0], fac["K1"])
    s.py = kick(s.py, g[1], fac["K1"])
    s.pz = kick(s.pz, g[2], fac["K1"])
    rec = lightcone_records(s, x_obs, fac["a0"], fac["a1"], fac["D"], fac["chi2_0"], fac["chi2_1"],
                            solve=solve, limit=lc_limit)
    s.x = drift(s.x, s.px, fac["D"], s.L)
    s.y = drift(s.y, s.py, fac["D"], s.L)
    s.z = drift(s.z, s.pz, fac["D"], s.L)
    cres = None
    if coarsen_params is not None:
        extra = {}
        if coarsen_params.get("alpha_dyn") is not None:
            extra = {"g": g, "Gm0": box.G * box.m0}
        out, group_of, nm = coarsen(s, x_obs, **coarsen_params, **extra)
        cres = (out, group_of, nm)
        for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
            setattr(s, k, out[k])
    gn = total_force(s.x, s.y, s.z, s.mult, box, ng, r_s, r_cut)
    s.px = kick(s.px, gn[0], fac["K2"])
    s.py = kick(s.py, gn[1], fac["K2"])
    s.pz = kick(s.pz, gn[2], fac["K2"])
    return s, gn, rec, cres


# ======================================================================================
# Individual power-of-two time steps (Sec. 2.1) with DZS only at global steps and the
# out-of-lightcone limiter (Sec. 2.2): a block-step kick-drift-kick inside one global step.
#
# Readings: the global step [a0, a1] is cut into S = 2^B sub-steps of equal length in ln a;
# a particle in bin b steps over 2^(B-b) sub-steps, its kicks reaching the midpoint of its own
# step in ln a (so B = 0 is the plain step).  Bins are set at the start of the global step
# from the accelerations held then: the step allowed is delta = sqrt(C eps / |g|), with
# C = 2 eta a0^3 H(a0)^2 (a constant acceleration moves a particle by eta eps over delta) and
# eps = eps0 mult^(1/3); the bin is the smallest b <= B with ln(a1/a0) 2^-b <= delta.
# Limiter: a particle outside the lightcone sphere (|x - x_obs| >= R_lim, minimum image)
# takes at most the largest bin held inside (no limit when nothing is inside).  Every
# particle that ends a step at a sub-step boundary gets its new force there (the full PM +
# short-range force).  DZS acts once every particle is synchronised at a1 (after the closing
# kicks, so the merged momenta are all taken at a1), and the merged particles' force is then
# computed anew (a state that merged nothing keeps its forces).
# ======================================================================================

def hier_bins(ps, g, box: Box, a0, a1, max_bin, eta, x_obs=None, R_lim=None, om=OMEGA_M):
    """Power-of-two bins of the particles for the global step a0 -> a1 (see above)."""
    H = H0 * math.sqrt(om / (a0 * a0 * a0) + (1.0 - om))
    C = 2.0 * eta * (a0 * a0 * a0) * (H * H)
    Dl = math.log(a1 / a0)
    g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2]
    gn = np.sqrt(g2)
    eps = box.eps0 * np.cbrt(np.asarray(ps.mult, np.float64))
    with np.errstate(divide="ignore"):
        delta = np.where(gn > 0, np.sqrt(C * eps / np.where(gn > 0, gn, 1.0)), np.inf)
    bins = np.zeros(ps.n, np.int64)
    for b in range(max_bin):
        bins[(bins == b) & (math.ldexp(Dl, -b) > delta)] += 1
    if R_lim is not None and x_obs is not None and ps.n:
        d = [min_image(getattr(ps, k) - x_obs[i], ps.L) for i, k in enumerate(("x", "y", "z"))]
        inside = np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) < R_lim
        if inside.any():
            cap = int(bins[inside].max())
            bins[~inside] = np.minimum(bins[~inside], cap)
    return bins


def hier_grid(a0, a1, max_bin):
    """Half-sub-step grid u_k, k = 0 .. 2 S, uniform in ln a from a0 to a1 (ends exact)."""
    S = 1 << max_bin
    la0, Dl = math.log(a0), math.log(a1 / a0)
    u = [math.exp(la0 + Dl * k / (2 * S)) for k in range(2 * S + 1)]
    u[0], u[-1] = a0, a1
    return u


def kdk_step_hier(ps, g, box: Box, a0, a1, max_bin, eta, ng, r_s, r_cut, x_obs, R_lim=None,
                  coarsen_params=None, solve=False, bins=None):
    """One global step a0 -> a1 with individual power-of-two steps.  Returns (new state, g
    (3, n) at a1, lightcone records of every sub-drift, coarsening result or None, bins)."""
    s = ps.copy()
    g = np.array(g, np.float64, copy=True)
    if bins is None:
        bins = hier_bins(s, g, box, a0, a1, max_bin, eta, x_obs, R_lim)
    S = 1 << max_bin
    u = hier_grid(a0, a1, max_bin)
    chi2 = [0.0 if uk >= 1.0 else chi(uk) ** 2 for uk in u]
    records, cres = [], None
    for j in range(S):
        for b in range(max_bin + 1):
            L = 1 << (max_bin - b)
            if j % L == 0:
                sel = bins == b
                if sel.any():
                    K = kick_factor(u[2 * j], u[2 * j + L])
                    s.px[sel] = kick(s.px[sel], g[0, sel], K)
                    s.py[sel] = kick(s.py[sel], g[1, sel], K)
                    s.pz[sel] = kick(s.pz[sel], g[2, sel], K)
        D = drift_factor(u[2 * j], u[2 * j + 2])
        records.append(lightcone_records(s, x_obs, u[2 * j], u[2 * j + 2], D, chi2[2 * j],
                                         chi2[2 * j + 2], solve=solve))
        s.x = drift(s.x, s.px, D, s.L)
        s.y = drift(s.y, s.py, D, s.L)
        s.z = drift(s.z, s.pz, D, s.L)
        jn = j + 1
        active = np.array([(jn % (1 << (max_bin - int(b)))) == 0 for b in bins], bool)
        if not active.any():
            continue
        gn = total_force(s.x, s.y, s.z, s.mult, box, ng, r_s, r_cut)
        g[:, active] = gn[:, active]
        for b in range(max_bin + 1):
            L = 1 << (max_bin - b)
            if jn % L == 0:
                sel = (bins == b) & active
                if sel.any():
                    K = kick_factor(u[2 * jn - L], u[2 * jn])
                    s.px[sel] = kick(s.px[sel], g[0, sel], K)
                    s.py[sel] = kick(s.py[sel], g[1, sel], K)
                    s.pz[sel] = kick(s.pz[sel], g[2, sel], K)
    if coarsen_params is not None:
        extra = {}
        if coarsen_params.get("alpha_dyn") is not None:
            extra = {"g": g, "Gm0": box.G * box.m0}
        out, group_of, nm = coarsen(s, x_obs, **coarsen_params, **extra)
        cres = (out, group_of, nm)
        for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
            setattr(s, k, out[k])
        if nm > 0:
            g = total_force(s.x, s.y, s.z, s.mult, box, ng, r_s, r_cut)
        else:
            g2 = np.empty_like(g)
            g2[:, group_of] = g
            g = g2
    return s, g, records, cres, bins


# ======================================================================================
# Individual time steps with the long-range force on the global step only (Sec. 2.1: the
# TreePM split carried into time, as the paper's code integrates its PM force with the
# largest step and the tree force with the individual ones).
#
# Reading: the state's g on entry is the total force at a0 (PM + short range, as every step
# leaves it).  The PM force is computed at a0, and the short-range part of the entry force
# is g - g_PM(a0).  The global step opens with a long-range half-kick g_PM(a0) K(a0, a_h)
# for every particle (a_h = sqrt(a0 a1), the step's midpoint in ln a), then runs the
# sub-step schedule of kdk_step_hier with the short-range force alone (kicks, drifts,
# lightcone tests and the short-range force of the particles that end a step at a sub-step
# boundary, computed on every particle's current position), and closes with the PM force at
# a1 and the half-kick g_PM(a1) K(a_h, a1) after the last short-range kicks.  The force left
# in the state is g_PM(a1) + g_SR(a1) (every particle ends a step at a1).  DZS at a1 as in
# kdk_step_hier, then a new total force if anything merged.  The bins come from |g| at a0.
# ======================================================================================

def kdk_step_hier_split(ps, g, box: Box, a0, a1, max_bin, eta, ng, r_s, r_cut, x_obs,
                        R_lim=None, coarsen_params=None, solve=False, bins=None):
    """One global step a0 -> a1: long-range kicks on the global step, short-range kicks on
    individual power-of-two steps.  Returns (new state, g (3, n) at a1, lightcone records of
    every sub-drift, coarsening result or None, bins)."""
    s = ps.copy()
    g = np.array(g, np.float64, copy=True)
    if bins is None:
        bins = hier_bins(s, g, box, a0, a1, max_bin, eta, x_obs, R_lim)
    S = 1 << max_bin
    u = hier_grid(a0, a1, max_bin)
    chi2 = [0.0 if uk >= 1.0 else chi(uk) ** 2 for uk in u]
    g_pm = pm_force(s.x, s.y, s.z, s.mult, box, ng, r_s)
    g_sr = g - g_pm
    K = kick_factor(a0, u[S])
    s.px = kick(s.px, g_pm[0], K)
    s.py = kick(s.py, g_pm[1], K)
    s.pz = kick(s.pz, g_pm[2], K)
    records, cres = [], None
    for j in range(S):
        for b in range(max_bin + 1):
            Lb = 1 << (max_bin - b)
            if j % Lb == 0:
                sel = bins == b
                if sel.any():
                    K = kick_factor(u[2 * j], u[2 * j + Lb])
                    s.px[sel] = kick(s.px[sel], g_sr[0, sel], K)
                    s.py[sel] = kick(s.py[sel], g_sr[1, sel], K)
                    s.pz[sel] = kick(s.pz[sel], g_sr[2, sel], K)
        D = drift_factor(u[2 * j], u[2 * j + 2])
        records.append(lightcone_records(s, x_obs, u[2 * j], u[2 * j + 2], D, chi2[2 * j],
                                         chi2[2 * j + 2], solve=solve))
        s.x = drift(s.x, s.px, D, s.L)
        s.y = drift(s.y, s.py, D, s.L)
        s.z = drift(s.z, s.pz, D, s.L)
        jn = j + 1
        active = np.array([(jn % (1 << (max_bin - int(b)))) == 0 for b in bins], bool)
        if not active.any():
            continue
        idx = np.nonzero(active)[0]
        g_sr[:, idx] = short_range(s.x, s.y, s.z, s.mult, box, r_s, r_cut, targets=idx)
        for b in range(max_bin + 1):
            Lb = 1 << (max_bin - b)
            if jn % Lb == 0:
                sel = (bins == b) & active
                if sel.any():
                    K = kick_factor(u[2 * jn - Lb], u[2 * jn])
                    s.px[sel] = kick(s.px[sel], g_sr[0, sel], K)
                    s.py[sel] = kick(s.py[sel], g_sr[1, sel], K)
                    s.pz[sel] = kick(s.pz[sel], g_sr[2, sel], K)
    g_pm = pm_force(s.x, s.y, s.z, s.mult, box, ng, r_s)
    K = kick_factor(u[S], a1)
    s.px = kick(s.px, g_pm[0], K)
    s.py = kick(s.py, g_pm[1], K)
    s.pz = kick(s.pz, g_pm[2], K)
    g = g_pm + g_sr
    if coarsen_params is not None:
        extra = {}
        if coarsen_params.get("alpha_dyn") is not None:
            extra = {"g": g, "Gm0": box.G * box.m0}
        out, group_of, nm = coarsen(s, x_obs, **coarsen_params, **extra)
        cres = (out, group_of, nm)
        for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
            setattr(s, k, out[k])
        if nm > 0:
            g = total_force(s.x, s.y, s.z, s.mult, box, ng, r_s, r_cut)
        else:
            g2 = np.empty_like(g)
            g2[:, group_of] = g
            g = g2
    return s, g, records, cres, bins

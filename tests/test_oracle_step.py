"""Pins for the oracle's cosmology, kick/drift and lightcone crossing.

* K, D and chi against closed forms: Einstein-de Sitter elementary integrals, and for flat
  LCDM the Gauss hypergeometric antiderivative of a^(s-1) (1 + r a^3)^(-1/2);
* zero force: the drift is exactly x0 + p D, wrapped;
* linear growth: a single Zel'dovich plane wave evolved with the oracle's full TreePM force
  and KDK integrator grows as the linear growth factor (from the growth ODE, solved here
  independently);
* lightcone: with p = 0 the crossing is at chi(a) = |d|, i.e. a = chi^-1(|d|) (inverted here
  on the hypergeometric closed form); over a sequence of steps every particle inside the
  initial sphere is emitted exactly once.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq
from scipy.special import hyp2f1

import dzs_ics
import oracle

OM = 0.3
R = (1 - OM) / OM


def _F(a, s):
    return a ** s / s * hyp2f1(0.5, s / 3.0, 1.0 + s / 3.0, -R * a ** 3)


def chi_closed(a):
    return oracle.C_LIGHT / oracle.H0 / math.sqrt(OM) * (_F(1.0, 0.5) - _F(a, 0.5))


def test_eds_closed_forms():
    for a0, a1 in ((0.02, 0.025), (0.3, 0.5), (0.9, 1.0)):
        K = oracle.kick_factor(a0, a1, om=1.0)
        D = oracle.drift_factor(a0, a1, om=1.0)
        assert abs(K - 2 * (math.sqrt(a1) - math.sqrt(a0)) / oracle.H0) <= 1e-14 * K
        assert abs(D - 2 * (a0 ** -0.5 - a1 ** -0.5) / oracle.H0) <= 1e-14 * D
    for a in (0.02, 0.5, 0.99):
        c = oracle.chi(a, om=1.0)
        assert abs(c - 2 * oracle.C_LIGHT / oracle.H0 * (1 - math.sqrt(a))) <= 1e-14 * c


@pytest.mark.parametrize("a0,a1", [(0.02, 0.02 * math.exp(0.07824)), (0.4, 0.45), (0.9247, 1.0)])
def test_lcdm_hypergeometric_closed_forms(a0, a1):
    K = oracle.kick_factor(a0, a1)
    D = oracle.drift_factor(a0, a1)
    Kc = (_F(a1, 0.5) - _F(a0, 0.5)) / (oracle.H0 * math.sqrt(OM))
    Dc = (_F(a1, -0.5) - _F(a0, -0.5)) / (oracle.H0 * math.sqrt(OM))
    assert abs(K - Kc) <= 1e-13 * K
    assert abs(D - Dc) <= 1e-13 * D
    for a in (a0, a1):
        if a < 1:
            assert abs(oracle.chi(a) - chi_closed(a)) <= 1e-13 * chi_closed(a)


def test_zero_force_drift_is_exact():
    ps = dzs_ics.uniform_random(1000, 64.0, seed=1, vel=800.0)
    D = oracle.drift_factor(0.5, 0.55)
    x1 = oracle.drift(ps.x, ps.px, D, ps.L)
    raw = ps.x + ps.px * D
    expect = raw - ps.L * np.floor(raw / ps.L)
    expect[expect >= ps.L] = 0.0
    assert np.array_equal(x1, expect)
    assert np.all((x1 >= 0) & (x1 < ps.L))


def _linear_growth(a_grid):
    """Growing mode of D'' + (3/a + E'/E) D' = 1.5 om D / (a^5 E^2), from D = a at a -> 0."""
    def E(a):
        return math.sqrt(OM / a ** 3 + 1 - OM)

    def rhs(a, y):
        Ea = E(a)
        dE = -1.5 * OM / a ** 4 / Ea
        return [y[1], -(3 / a + dE / Ea) * y[1] + 1.5 * OM / (a ** 5 * Ea ** 2) * y[0]]
    a_start = 1e-3
    sol = solve_ivp(rhs, (a_start, max(a_grid)), [a_start, 1.0], rtol=1e-12, atol=1e-15,
                    dense_output=True)
    return sol


@pytest.mark.slow
def test_zeldovich_plane_wave_grows_linearly():
    n_side, L = 16, 64.0
    lam = L / n_side
    ng = 2 * n_side
    r_s = 1.25 * L / ng
    ps = dzs_ics.lattice(n_side, L)
    box = oracle.Box(L=L, m0=dzs_ics.particle_mass(L, ps.n), eps0=lam / 40)
    k = 2 * math.pi / L
    A0 = 0.05 * lam
    a_i, a_f, n_steps = 0.02, 0.2, 24
    sol = _linear_growth([a_f])
    D_i, dD_i = sol.sol(a_i)
    f_i = a_i * dD_i / D_i
    q = ps.x.copy()
    psi = A0 * np.sin(k * q)
    ps.x = oracle.wrap(q + psi, L)
    H_i = oracle.H0 * math.sqrt(OM / a_i ** 3 + 1 - OM)
    ps.px = a_i ** 2 * H_i * f_i * psi
    g = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, box, ng, r_s, 4.5 * r_s)
    a_grid = np.exp(np.linspace(math.log(a_i), math.log(a_f), n_steps + 1))
    for n in range(n_steps):
        a0, a1 = a_grid[n], a_grid[n + 1]
        ah = math.sqrt(a0 * a1)
        fac = {"a0": a0, "a1": a1, "K1": oracle.kick_factor(a0, ah),
               "D": oracle.drift_factor(a0, a1), "K2": oracle.kick_factor(ah, a1),
               "chi2_0": 1e30, "chi2_1": 1e30}
        ps, g, _, _ = oracle.kdk_step(ps, g, box, fac, ng, r_s, 4.5 * r_s, [0.0, 0.0, 0.0],
                                      solve=False)
    disp = oracle.min_image(ps.x - q, L)
    amp = 2 * np.mean(disp * np.sin(k * q))     # projection on the mode
    expect = A0 * sol.sol(a_f)[0] / D_i
    assert abs(amp / expect - 1) < 1e-3
    # transverse motion stays zero
    assert np.abs(oracle.min_image(ps.y - dzs_ics.lattice(n_side, L).y, L)).max() < 1e-9 * lam


def test_lightcone_static_particle_crosses_at_inverse_distance():
    L = 4000.0
    rs = np.array([520.0, 800.0, 1310.0, 2900.0])  # inside [chi(a1), chi(a0)]
    a0, a1 = 0.4, 0.85
    c0, c1 = oracle.chi(a0), oracle.chi(a1)
    D = oracle.drift_factor(a0, a1)
    for r in rs:
        d0 = np.array([r, 0.0, 0.0])
        ac = oracle.crossing_time(d0, np.zeros(3), a0, a1)
        a_ref = brentq(lambda a: chi_closed(a) - r, 0.05, 0.9999, xtol=1e-16, rtol=8.9e-16)
        assert abs(ac - a_ref) <= 1e-12
        mask, *_ = oracle.lightcone_select(np.array([r]), np.array([0.0]), np.array([0.0]),
                                           np.zeros(1), np.zeros(1), np.zeros(1), L,
                                           [0.0, 0.0, 0.0], D, c0 * c0, c1 * c1)
        assert mask[0] == (c1 <= r < c0)


def test_lightcone_emits_each_static_particle_once():
    L = 3000.0
    ps = dzs_ics.uniform_random(4000, L, seed=12)
    a_grid = np.exp(np.linspace(math.log(0.5), 0.0, 13))
    chis = [oracle.chi(a) if a < 1 else 0.0 for a in a_grid]
    counts = np.zeros(ps.n, np.int64)
    for n in range(len(a_grid) - 1):
        D = oracle.drift_factor(a_grid[n], a_grid[n + 1])
        mask, *_ = oracle.lightcone_select(ps.x, ps.y, ps.z, ps.px, ps.py, ps.pz, L,
                                           [0.0, 0.0, 0.0], D, chis[n] ** 2, chis[n + 1] ** 2)
        counts += mask
    d = np.sqrt(sum(oracle.min_image(c, L) ** 2 for c in (ps.x, ps.y, ps.z)))
    inside = (d > 0) & (d < chis[0])
    assert np.all(counts[inside] == 1)
    assert np.all(counts[~inside] == 0)


def test_lightcone_moving_particles_record_consistency():
    """A moving particle's record: |d(a_x)| = chi(a_x) at the solved crossing, on the drift line."""
    L = 2000.0
    ps = dzs_ics.uniform_random(3000, L, seed=5, vel=1500.0)
    a0, a1 = 0.7, 0.74
    fac = oracle.step_factors(a0, a1)
    rec = oracle.lightcone_records(ps, [0.0, 0.0, 0.0], a0, a1, fac["D"], fac["chi2_0"],
                                   fac["chi2_1"])
    assert rec["id"].size > 5
    for r in range(rec["id"].size):
        ac = rec["a_cross"][r]
        assert a0 <= ac <= a1
        dn = np.linalg.norm(rec["d"][r])
        assert abs(dn - chi_closed(ac)) <= 1e-9 * dn


def test_lightcone_particle_moving_through_the_antipode_is_emitted_once():
    """A particle that drifts across the face of the periodic cell opposite the observer just
    as the sphere reaches it: its minimum-image distance shrinks from 49.9 to 49.9 via 50.
    Unwrapped, the end-of-drift distance would be 50.1 (outside a sphere of radius 50): it
    would be emitted in the first drift and again in the second, when the sphere passes its
    true distance.  Each particle crosses the past lightcone once (Sec. 3.1.3), so the test at
    the end of a drift must be the test at the start of the next."""
    L = 100.0
    x, y, z = np.array([49.9]), np.array([0.0]), np.array([0.0])
    px, py, pz = np.array([1.0]), np.array([0.0]), np.array([0.0])
    D = 0.2                          # one drift moves the particle by 0.2 along x
    chis = [50.05, 50.0, 49.6]
    emitted = 0
    for n in range(2):
        mask, _, f0, f1 = oracle.lightcone_select(x, y, z, px, py, pz, L, [0.0, 0.0, 0.0], D,
                                                  chis[n] ** 2, chis[n + 1] ** 2)
        emitted += int(mask[0])
        x = oracle.drift(x, px, D, L)
        # the next drift starts from exactly this end-of-drift test value
        d_next = oracle.min_image(x, L)
        assert float(d_next[0] ** 2 - chis[n + 1] ** 2) == float(f1[0])
    assert emitted == 1

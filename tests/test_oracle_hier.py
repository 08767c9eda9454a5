"""Pins for the oracle's individual power-of-two time steps (paper Sec. 2.1; DZS at global
steps and the out-of-lightcone limiter of Sec. 2.2).

* B = 0 is the plain kick-drift-kick step;
* every particle held in one bin b is 2^b plain steps on the sub-step grid;
* mixed bins on a Zel'dovich plane wave (bins that really differ across the wave) stay with
  the finest-step run, far closer than the coarsest-step run; all grow at the linear rate;
* the bin rule against a closed form (ceil of log2) away from bin edges; the limiter caps
  particles outside the sphere at the largest bin inside, and does nothing with nobody inside.
"""
import math

import numpy as np
import pytest

import dzs_ics
import oracle
from test_oracle_step import OM, _linear_growth


def _box(n_side, L):
    ps = dzs_ics.zeldovich(n_side, L, 0.05, seed=77, spectrum="powerlaw")
    box = oracle.Box(L=L, m0=dzs_ics.particle_mass(L, ps.n), eps0=L / n_side / 40)
    return ps, box


def _plain_steps(ps, g, box, u, ng, r_s, r_cut, stride):
    """Plain KDK steps between the grid points u[0], u[stride], u[2 stride], ..."""
    s = ps
    for k in range(0, len(u) - 1, stride):
        a0, ah, a1 = u[k], u[k + stride // 2], u[k + stride]
        fac = {"a0": a0, "a1": a1, "K1": oracle.kick_factor(a0, ah),
               "D": oracle.drift_factor(a0, a1), "K2": oracle.kick_factor(ah, a1),
               "chi2_0": 1e30, "chi2_1": 1e30}
        s, g, _, _ = oracle.kdk_step(s, g, box, fac, ng, r_s, r_cut, [0.0, 0.0, 0.0],
                                     solve=False)
    return s, g


def _close(a, b, tol):
    return np.abs(a - b).max() <= tol * (np.abs(b).max() + 1e-300)


def test_single_bin_zero_is_the_plain_step():
    ps, box = _box(12, 50.0)
    ng, r_s = 24, 1.25 * 50.0 / 24
    g = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, box, ng, r_s, 4.5 * r_s)
    a0, a1 = 0.05, 0.06
    sh, gh, _, _, bins = oracle.kdk_step_hier(ps, g, box, a0, a1, 0, 0.025, ng, r_s,
                                              4.5 * r_s, [0.0, 0.0, 0.0])
    assert np.all(bins == 0)
    sp, gp = _plain_steps(ps, g, box, oracle.hier_grid(a0, a1, 0), ng, r_s, 4.5 * r_s, 2)
    for k in ("x", "y", "z", "px", "py", "pz"):
        assert _close(getattr(sh, k), getattr(sp, k), 1e-13), k
    assert _close(gh, gp, 1e-12)


@pytest.mark.parametrize("b", [1, 2])
def test_one_shared_bin_is_plain_substeps(b):
    ps, box = _box(10, 40.0)
    ng, r_s = 20, 1.25 * 40.0 / 20
    g = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, box, ng, r_s, 4.5 * r_s)
    a0, a1, B = 0.05, 0.07, 2
    bins = np.full(ps.n, b)
    sh, gh, _, _, _ = oracle.kdk_step_hier(ps, g, box, a0, a1, B, 0.025, ng, r_s, 4.5 * r_s,
                                           [0.0, 0.0, 0.0], bins=bins)
    u = oracle.hier_grid(a0, a1, B)
    sp, gp = _plain_steps(ps, g, box, u, ng, r_s, 4.5 * r_s, 2 * (1 << (B - b)))
    for k in ("x", "y", "z", "px", "py", "pz"):
        assert _close(getattr(sh, k), getattr(sp, k), 1e-12), k


def test_mixed_bins_track_the_finest_steps_on_a_plane_wave():
    """A Zel'dovich plane wave spreads the particles over the bins (|g| follows the wave).
    The mixed-bin run stays with the run that gives every particle the finest step, far
    closer than the run that gives every particle the whole global step, and all three grow
    the wave at the linear rate (an independent ODE) to the accuracy of the force."""
    n_side, L = 16, 64.0
    lam = L / n_side
    ng = 2 * n_side
    r_s = 1.25 * L / ng
    k = 2 * math.pi / L
    A0 = 0.05 * lam
    a_i, a_f, n_steps = 0.02, 0.2, 12
    sol = _linear_growth([a_f])
    D_i, dD_i = sol.sol(a_i)
    a_grid = np.exp(np.linspace(math.log(a_i), math.log(a_f), n_steps + 1))

    def run(fixed_bin):
        ps = dzs_ics.lattice(n_side, L)
        box = oracle.Box(L=L, m0=dzs_ics.particle_mass(L, ps.n), eps0=lam / 40)
        q = ps.x.copy()
        psi = A0 * np.sin(k * q)
        ps.x = oracle.wrap(q + psi, L)
        H_i = oracle.H0 * math.sqrt(OM / a_i ** 3 + 1 - OM)
        ps.px = a_i ** 2 * H_i * (a_i * dD_i / D_i) * psi
        g = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, box, ng, r_s, 4.5 * r_s)
        seen = set()
        for n in range(n_steps):
            bins = None if fixed_bin is None else np.full(ps.n, fixed_bin)
            ps, g, _, _, b = oracle.kdk_step_hier(ps, g, box, a_grid[n], a_grid[n + 1], 2,
                                                  0.01, ng, r_s, 4.5 * r_s, [0.0, 0.0, 0.0],
                                                  bins=bins)
            seen |= set(np.unique(b).tolist())
        disp = oracle.min_image(ps.x - q, L)
        return 2 * np.mean(disp * np.sin(k * q)) / (A0 * sol.sol(a_f)[0] / D_i), seen

    coarse, _ = run(0)
    fine, _ = run(2)
    mixed, seen = run(None)
    assert len(seen) >= 2, "the wave should spread the particles over several bins"
    assert abs(mixed - fine) <= 0.1 * abs(coarse - fine)
    for v in (coarse, fine, mixed):
        assert abs(v - 1) < 1e-2


def test_bin_rule_and_limiter():
    L = 100.0
    ps = dzs_ics.uniform_random(4000, L, seed=5)
    ps = dzs_ics.merged_state(ps, seed=6, max_mult=27)
    box = oracle.Box(L=L, m0=1.0, eps0=0.05)
    g = dzs_ics.rng(8).standard_normal((3, ps.n)) * np.exp(dzs_ics.rng(9).uniform(3, 17, ps.n))
    a0, a1, B, eta = 0.3, 0.33, 5, 0.025
    bins = oracle.hier_bins(ps, g, box, a0, a1, B, eta)
    H = oracle.H0 * math.sqrt(OM / a0 ** 3 + 1 - OM)
    delta = np.sqrt(2 * eta * a0 ** 3 * H ** 2 * box.eps0 * np.cbrt(ps.mult)
                    / np.linalg.norm(g, axis=0))
    x = np.log2(math.log(a1 / a0) / delta)
    far = np.abs(x - np.round(x)) > 1e-9
    ref = np.clip(np.ceil(x), 0, B).astype(int)
    assert np.array_equal(bins[far], ref[far])
    assert len(np.unique(bins)) == B + 1
    # limiter: outside R_lim capped at the largest bin inside
    xo, R = [10.0, 20.0, 30.0], 15.0
    lb = oracle.hier_bins(ps, g, box, a0, a1, B, eta, x_obs=xo, R_lim=R)
    d = [oracle.min_image(getattr(ps, k) - xo[i], L) for i, k in enumerate("xyz")]
    inside = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2) < R
    cap = bins[inside].max()
    assert np.array_equal(lb[inside], bins[inside])
    assert np.array_equal(lb[~inside], np.minimum(bins[~inside], cap))
    # nobody inside: no limit
    assert np.array_equal(oracle.hier_bins(ps, g, box, a0, a1, B, eta, x_obs=xo, R_lim=0.0),
                          bins)


# ---- the long-range force on the global step only (kdk_step_hier_split) -----------------

def test_split_step_with_one_bin_is_the_plain_step():
    """B = 0: the long-range half-kicks and the short-range kicks of the one sub-step make up
    the plain step's kicks (the PM force at a0 and a1, the short range at a0 and a1)."""
    ps, box = _box(12, 50.0)
    ng, r_s = 24, 1.25 * 50.0 / 24
    g = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, box, ng, r_s, 4.5 * r_s)
    a0, a1 = 0.05, 0.06
    sh, gh, _, _, bins = oracle.kdk_step_hier_split(ps, g, box, a0, a1, 0, 0.025, ng, r_s,
                                                    4.5 * r_s, [0.0, 0.0, 0.0])
    assert np.all(bins == 0)
    sp, gp = _plain_steps(ps, g, box, oracle.hier_grid(a0, a1, 0), ng, r_s, 4.5 * r_s, 2)
    for k in ("x", "y", "z", "px", "py", "pz"):
        assert _close(getattr(sh, k), getattr(sp, k), 1e-13), k
    assert _close(gh, gp, 1e-12)


def test_split_step_without_short_range_pairs_ignores_the_bins():
    """With no pair inside r_cut the force is the PM force alone, which the split step
    applies on the global step only: any spread of bins gives the plain step (the sub-drifts
    add up to the step's drift)."""
    ps, box = _box(12, 50.0)
    ng, r_s = 24, 1.25 * 50.0 / 24
    r_cut = 1e-4 * 50.0 / 12
    g = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, box, ng, r_s, r_cut)
    a0, a1, B = 0.05, 0.07, 2
    bins = np.arange(ps.n) % (B + 1)
    sh, gh, _, _, _ = oracle.kdk_step_hier_split(ps, g, box, a0, a1, B, 0.025, ng, r_s, r_cut,
                                                 [0.0, 0.0, 0.0], bins=bins)
    sp, gp = _plain_steps(ps, g, box, oracle.hier_grid(a0, a1, 0), ng, r_s, r_cut, 2)
    for k in ("x", "y", "z", "px", "py", "pz"):
        assert _close(getattr(sh, k), getattr(sp, k), 1e-12), k
    assert _close(gh, gp, 1e-12)
    # the same bins in the step that recomputes the whole force at every sub-step differ
    so, _, _, _, _ = oracle.kdk_step_hier(ps, g, box, a0, a1, B, 0.025, ng, r_s, r_cut,
                                          [0.0, 0.0, 0.0], bins=bins)
    assert not _close(so.px, sp.px, 1e-9)


def test_split_step_grows_a_plane_wave_at_the_linear_rate():
    """Mixed bins with the long-range force on the global step follow the linear growth of a
    Zel'dovich plane wave (an independent ODE) and stay with the run that puts every particle
    in the finest bin."""
    n_side, L = 16, 64.0
    lam = L / n_side
    ng = 2 * n_side
    r_s = 1.25 * L / ng
    k = 2 * math.pi / L
    A0 = 0.05 * lam
    a_i, a_f, n_steps = 0.02, 0.2, 12
    sol = _linear_growth([a_f])
    D_i, dD_i = sol.sol(a_i)
    a_grid = np.exp(np.linspace(math.log(a_i), math.log(a_f), n_steps + 1))

    def run(fixed_bin):
        ps = dzs_ics.lattice(n_side, L)
        box = oracle.Box(L=L, m0=dzs_ics.particle_mass(L, ps.n), eps0=lam / 40)
        q = ps.x.copy()
        psi = A0 * np.sin(k * q)
        ps.x = oracle.wrap(q + psi, L)
        H_i = oracle.H0 * math.sqrt(OM / a_i ** 3 + 1 - OM)
        ps.px = a_i ** 2 * H_i * (a_i * dD_i / D_i) * psi
        g = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, box, ng, r_s, 4.5 * r_s)
        seen = set()
        for n in range(n_steps):
            bins = None if fixed_bin is None else np.full(ps.n, fixed_bin)
            ps, g, _, _, b = oracle.kdk_step_hier_split(ps, g, box, a_grid[n], a_grid[n + 1],
                                                        2, 0.01, ng, r_s, 4.5 * r_s,
                                                        [0.0, 0.0, 0.0], bins=bins)
            seen |= set(np.unique(b).tolist())
        disp = oracle.min_image(ps.x - q, L)
        return 2 * np.mean(disp * np.sin(k * q)) / (A0 * sol.sol(a_f)[0] / D_i), seen

    fine, _ = run(2)
    mixed, seen = run(None)
    assert len(seen) >= 2
    assert abs(mixed - fine) <= 2e-3
    for v in (fine, mixed):
        assert abs(v - 1) < 1e-2

"""Pins for the oracle's dynamical DZS criterion (paper Sec. 2.2.1: eq. 2 made node-centric
with eq. 3, and the previous acceleration replaced by its minimum inside the lightcone).

* worked example: a two-particle node at D_n = 1/4 with dyadic G m0, l_k and a_min, where the
  merge threshold alpha = 1/2 is exact, so the strict inequality is checked at equality and on
  both sides; the in-lightcone minimum ignores particles outside R_lc + b and on its boundary;
* exact-math brute force: per-level cube bucketing with exact rationals for the centres of
  mass, distances and accelerations and 50-digit decimals for the square and fourth roots;
* dimensional analysis: scaling lengths by 2 and accelerations by 1/4, or G m0 and the
  accelerations by 2, leaves every decision unchanged (catches a wrong power of l_k or D_n);
* limits and order: alpha = 0 merges nothing; a huge alpha reduces to "every node with D_n > 0",
  i.e. the geometric criterion at an infinite opening angle; groups nest as alpha grows.
"""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import dzs_ics
import oracle


def _mi(d, L):
    if d >= L / 2:
        return d - L
    if d < -L / 2:
        return d + L
    return d


def _groups(ps, res, group_of):
    """{frozenset(member ids) -> output index} for the merged outputs."""
    n_out = res["x"].shape[0]
    members = [[] for _ in range(n_out)]
    for i in range(ps.n):
        members[group_of[i]].append(int(ps.id[i]))
    return {frozenset(m): j for j, m in enumerate(members) if res["type"][j] == 1 and len(m) > 1}


def _state(points, L, g):
    n = len(points)
    p = np.asarray(points, np.float64).T
    z = np.zeros(n)
    ps = dzs_ics.ParticleSet(p[0].copy(), p[1].copy(), p[2].copy(), z.copy(), z.copy(), z.copy(),
                             np.ones(n, np.uint32), np.arange(n, dtype=np.uint32),
                             np.zeros(n, np.uint8), L)
    return ps, np.asarray(g, np.float64).T.copy()


# ------------------------------------------------------------------------------------------
# worked example with exact dyadic numbers
# ------------------------------------------------------------------------------------------

def _worked(alpha, inner_at=0.0625):
    """L = 1, observer at the origin, R_lc = 1/8, b = 0, k_min = 2 (l_2 = 1/4).
    Node: two unit particles at x = 5/16 and 7/16 on the x axis, centre of mass 3/8, so
    D = 3/8 - 1/8 = 1/4 and D^4 = 1/256.  With G m0 = 1/64 and K = 2 the left side is
    (1/64 * 2) * 1/16 = 1/512, so the node merges iff alpha a_min / 256 > 1/512.
    Particles inside: |g| = 1 at x = inner_at and |g| = 5 at x = 15/16 (min image -1/16).
    The node's own members have |g| = 1e-3 but lie outside the lightcone."""
    pts = [(0.3125, 0.0, 0.0), (0.4375, 0.0, 0.0), (inner_at, 0.0, 0.0), (0.9375, 0.0, 0.0)]
    g = [(1e-3, 0.0, 0.0), (0.0, -1e-3, 0.0), (0.0, 0.0, -1.0), (3.0, -4.0, 0.0)]
    ps, gg = _state(pts, 1.0, g)
    return ps, gg, oracle.coarsen(ps, [0.0, 0.0, 0.0], 0.125, 0.0, None, 2, alpha_dyn=alpha,
                                  g=gg, Gm0=1.0 / 64)


def test_worked_example_threshold_is_exact():
    for alpha, merges in ((0.4999999, False), (0.5, False), (0.5000001, True), (0.26, False),
                          (3.0, True)):
        ps, gg, (res, group_of, nm) = _worked(alpha)
        assert res["a_min"] == 1.0
        assert nm == (1 if merges else 0), alpha
        if merges:
            assert group_of[0] == group_of[1] and res["mult"][group_of[0]] == 2
            assert res["x"][group_of[0]] == 0.375
        assert group_of[2] != group_of[3]


def test_worked_example_inside_set_is_strict():
    # the |g| = 1 particle on the lightcone boundary (d = R_lc + b exactly) is not inside:
    # a_min becomes 5 and the threshold drops to alpha = 1/10
    ps, gg, (res, _, nm) = _worked(0.11, inner_at=0.125)
    assert res["a_min"] == 5.0 and nm == 1
    ps, gg, (res, _, nm) = _worked(0.1, inner_at=0.125)
    assert nm == 0
    assert oracle.a_min_lightcone(ps.x, ps.y, ps.z, gg, 1.0, [0, 0, 0], 0.125, 0.0) == 5.0
    # nobody inside: a_min = +inf and every node with D > 0 merges, whatever alpha > 0
    assert oracle.a_min_lightcone(ps.x, ps.y, ps.z, gg, 1.0, [0, 0, 0], 0.01, 0.0) == math.inf
    ps2, gg2 = _state([(0.3125, 0, 0), (0.4375, 0, 0)], 1.0, [(1, 0, 0), (0, 1, 0)])
    res, _, nm = oracle.coarsen(ps2, [0, 0, 0], 0.01, 0.0, None, 2, alpha_dyn=1e-300, g=gg2,
                                Gm0=1.0)
    assert res["a_min"] == math.inf and nm == 1


# ------------------------------------------------------------------------------------------
# exact-math brute force
# ------------------------------------------------------------------------------------------

def brute_dyn(ps, g, x_obs, R, b, k_min, alpha, Gm0):
    getcontext().prec = 50
    L = Fraction(ps.L)
    n = ps.n
    X = [[Fraction(float(v)) for v in arr] for arr in (ps.x, ps.y, ps.z)]
    M = [int(m) for m in ps.mult]
    xo = [Fraction(float(v)) for v in x_obs]
    Rb = Fraction(float(R)) + Fraction(float(b))
    best = None
    for i in range(n):
        dv = [_mi(X[d][i] - xo[d], L) for d in range(3)]
        if sum(v * v for v in dv) < Rb * Rb:
            g2 = sum(Fraction(float(g[d][i])) ** 2 for d in range(3))
            best = g2 if best is None or g2 < best else best
    if best is None:
        return None, {}, 0.0
    a_min = (Decimal(best.numerator) / Decimal(best.denominator)).sqrt()
    rhs0 = Decimal(float(alpha)) * a_min
    Rbd = Decimal(Rb.numerator) / Decimal(Rb.denominator)
    done = [False] * n
    groups = {}
    closest = math.inf
    for k in range(k_min, 22):
        side = 2 ** k
        l2 = (L / side) ** 2
        cubes = {}
        for i in range(n):
            if not done[i]:
                c = tuple(min(math.floor(X[d][i] * side / L), side - 1) for d in range(3))
                cubes.setdefault(c, []).append(i)
        if all(len(m) < 2 for m in cubes.values()):
            break
        for members in cubes.values():
            if len(members) < 2:
                continue
            K = sum(M[i] for i in members)
            com = [sum(M[i] * X[d][i] for i in members) / K for d in range(3)]
            dv = [_mi(com[d] - xo[d], L) for d in range(3)]
            d2 = dv[0] ** 2 + dv[1] ** 2 + dv[2] ** 2
            if not d2 > Rb * Rb:
                continue
            D = (Decimal(d2.numerator) / Decimal(d2.denominator)).sqrt() - Rbd
            lhs_f = Fraction(float(Gm0)) * K * l2
            lhs = Decimal(lhs_f.numerator) / Decimal(lhs_f.denominator)
            rhs = rhs0 * D ** 4
            closest = min(closest, float(abs(rhs - lhs) / lhs))
            if lhs < rhs:
                groups[frozenset(int(ps.id[i]) for i in members)] = K
                for i in members:
                    done[i] = True
    return float(a_min), groups, closest


@pytest.mark.parametrize("case", range(4))
def test_dynamical_matches_exact_math_bruteforce(case):
    L = [1.0, 100.0][case % 2]
    n = [800, 1600][case // 2]
    ps = dzs_ics.clustered_random(n, L, seed=400 + case, n_clumps=5, r_clump=L / 25)
    if case >= 2:
        ps = dzs_ics.merged_state(ps, seed=case)
    g = dzs_ics.rng(500 + case).standard_normal((3, n)) * (1.0 + case)
    x_obs = [0.0, 0.0, 0.0] if case % 2 == 0 else [0.3 * L, 0.7 * L, 0.1 * L]
    R, b, k_min = 0.15 * L, 0.02 * L, 2 + case % 2
    Gm0 = 1e-3 * L ** 2 * (1.0 + case) / n
    for alpha in (3e-3, 3e-2):
        res, group_of, nm = oracle.coarsen(ps, x_obs, R, b, None, k_min, alpha_dyn=alpha, g=g,
                                           Gm0=Gm0)
        a_min, ref, closest = brute_dyn(ps, g, x_obs, R, b, k_min, alpha, Gm0)
        assert closest > 1e-9, "a node sits on the threshold: choose another seed"
        assert abs(res["a_min"] - a_min) <= 1e-15 * a_min
        got = _groups(ps, res, group_of)
        assert set(got) == set(ref)
        assert all(int(res["mult"][j]) == ref[ids] for ids, j in got.items())
        assert nm == len(ref)
    assert nm > 3, "test case should exercise merging"


# ------------------------------------------------------------------------------------------
# dimensional analysis, limits, nesting
# ------------------------------------------------------------------------------------------

def _clustered(seed, n=6000, L=64.0):
    ps = dzs_ics.merged_state(dzs_ics.clustered_random(n, L, seed=seed, n_clumps=6), seed=seed)
    g = dzs_ics.rng(seed + 1).standard_normal((3, n))
    return ps, g


def _run(ps, g, alpha, Gm0, R=8.0, b=2.0, k_min=2, xo=(5.0, 9.0, 3.0)):
    return oracle.coarsen(ps, list(xo), R, b, None, k_min, alpha_dyn=alpha, g=g, Gm0=Gm0)


def test_decisions_invariant_under_exact_rescaling():
    ps, g = _clustered(31)
    alpha, Gm0 = 2e-3, 1e-3
    res, gof, nm = _run(ps, g, alpha, Gm0)
    assert nm > 50
    # lengths x 2 (positions, box, R_lc, b, observer) and accelerations x 1/4: G M l^2 / D^4
    # and alpha a_min both scale by 1/4 exactly
    ps2 = ps.copy()
    ps2.x, ps2.y, ps2.z, ps2.L = ps.x * 2, ps.y * 2, ps.z * 2, ps.L * 2
    res2, gof2, nm2 = _run(ps2, g / 4, alpha, Gm0, R=16.0, b=4.0, xo=(10.0, 18.0, 6.0))
    assert nm2 == nm and np.array_equal(gof, gof2) and res2["a_min"] == res["a_min"] / 4
    # G m0 x 2 and accelerations x 2
    res3, gof3, nm3 = _run(ps, g * 2, alpha, Gm0 * 2)
    assert nm3 == nm and np.array_equal(gof, gof3)
    # alpha x 2 and accelerations x 1/2
    res4, gof4, nm4 = _run(ps, g / 2, alpha * 2, Gm0)
    assert nm4 == nm and np.array_equal(gof, gof4)
    # but alpha x 2 alone changes the outcome
    res5, gof5, nm5 = _run(ps, g, alpha * 2, Gm0)
    assert res5["x"].shape[0] < res["x"].shape[0]


def test_limits_zero_and_huge_alpha():
    ps, g = _clustered(32)
    res, gof, nm = _run(ps, g, 0.0, 1e-3)
    assert nm == 0 and res["x"].shape[0] == ps.n
    # alpha a_min D^4 -> infinity: every node with D > 0 (and >= 2 members, k >= k_min) merges,
    # which is the geometric criterion with theta -> infinity (T_k -> R_lc + b)
    res, gof, nm = _run(ps, g, 1e300, 1e-3)
    geo, gof_g, nm_g = oracle.coarsen(ps, [5.0, 9.0, 3.0], 8.0, 2.0, 1e300, 2)
    assert nm == nm_g > 0 and np.array_equal(gof, gof_g)


def test_groups_nest_as_alpha_grows():
    ps, g = _clustered(33)
    prev_gof, prev_n = None, ps.n + 1
    for alpha in (1e-5, 1e-4, 1e-3, 1e-2, 1e-1):
        res, gof, nm = _run(ps, g, alpha, 1e-3)
        n_out = res["x"].shape[0]
        assert n_out <= prev_n
        if prev_gof is not None:
            # particles sharing an output at the smaller alpha still share one
            pairs = {}
            for i in range(ps.n):
                pairs.setdefault(prev_gof[i], set()).add(gof[i])
            assert all(len(v) == 1 for v in pairs.values())
        prev_gof, prev_n = gof, n_out
    assert prev_n < ps.n // 2

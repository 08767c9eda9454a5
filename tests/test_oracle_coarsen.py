"""Pins for the oracle's DZS coarsening (paper Sec. 2.2, 2.2.1; eqs. 1 and 3).

* brute force: an exact-rational (fractions) re-implementation of "each particle joins the
  shallowest level-k cube (k >= k_min, >= 2 members) whose centre of mass lies farther than
  R_lc + b + l_k / theta from the observer", on small random and clustered sets;
* closed forms: a lattice with every node outside the lightcone keeps (lambda/l_max)^3 of its
  particles — the 0.0157 bound the paper prints for l_max = 4 lambda, and the mass ratios 8 and
  64 it quotes for l_max = 2 and 4 lambda; nothing merges once R_lc + b >= sqrt(3)/2 L;
* invariants: exact mass conservation, momentum and centre-of-mass conservation to rounding,
  independence of the input order.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import dzs_ics
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=", 1)
            vals[k.strip()] = float(v)
    return vals


def _mi(d, L):
    if d >= L / 2:
        return d - L
    if d < -L / 2:
        return d + L
    return d


def brute_coarsen(ps, x_obs, R, b, theta, k_min):
    """Exact-rational reference: returns {frozenset(member ids): (K, com, mean p, min id)}."""
    L = Fraction(ps.L)
    n = ps.n
    X = [[Fraction(float(v)) for v in arr] for arr in (ps.x, ps.y, ps.z)]
    P = [[Fraction(float(v)) for v in arr] for arr in (ps.px, ps.py, ps.pz)]
    M = [int(m) for m in ps.mult]
    xo = [Fraction(float(v)) for v in x_obs]
    done = [False] * n
    groups = {}
    for k in range(k_min, 22):
        side = 2 ** k
        T = Fraction(float(R)) + Fraction(float(b)) + (L / side) / Fraction(float(theta))
        cubes = {}
        for i in range(n):
            if done[i]:
                continue
            c = tuple(min(math.floor(X[d][i] * side / L), side - 1) for d in range(3))
            cubes.setdefault(c, []).append(i)
        for members in cubes.values():
            if len(members) < 2:
                continue
            K = sum(M[i] for i in members)
            com = [sum(M[i] * X[d][i] for i in members) / K for d in range(3)]
            dv = [_mi(com[d] - xo[d], L) for d in range(3)]
            if dv[0] ** 2 + dv[1] ** 2 + dv[2] ** 2 > T * T:
                pm = [sum(M[i] * P[d][i] for i in members) / K for d in range(3)]
                ids = frozenset(int(ps.id[i]) for i in members)
                groups[ids] = (K, com, pm, min(ids))
                for i in members:
                    done[i] = True
    return groups


def oracle_groups(ps, res, group_of):
    n_out = res["x"].shape[0]
    members = [[] for _ in range(n_out)]
    for i in range(ps.n):
        members[group_of[i]].append(int(ps.id[i]))
    return {frozenset(m): j for j, m in enumerate(members) if len(m) > 1 or res["type"][j] == 1
            and ps.type[np.nonzero(ps.id == m[0])[0][0]] == 0}


@pytest.mark.parametrize("case", range(6))
def test_coarsen_matches_exact_rational_bruteforce(case):
    L = [1.0, 100.0, 256.0][case % 3]
    n = [600, 1500, 3000][case % 3]
    if case < 3:
        ps = dzs_ics.clustered_random(n, L, seed=100 + case, n_clumps=5, r_clump=L / 25)
    else:
        ps = dzs_ics.merged_state(dzs_ics.uniform_random(n, L, seed=200 + case, vel=100.0), seed=case)
    x_obs = [0.0, 0.0, 0.0] if case % 2 == 0 else [0.3 * L, 0.7 * L, 0.1 * L]
    R, b, theta, k_min = 0.12 * L, 0.02 * L, [0.5, 1.0, 2.0][case % 3], 2 + case % 2
    res, group_of, nm = oracle.coarsen(ps, x_obs, R, b, theta, k_min)
    ref = brute_coarsen(ps, x_obs, R, b, theta, k_min)
    assert nm == len(ref)
    assert nm > 3, "test case should exercise merging"
    # partition: every merged output particle's members equal one reference group
    n_out = res["x"].shape[0]
    members = [[] for _ in range(n_out)]
    for i in range(ps.n):
        members[group_of[i]].append(int(ps.id[i]))
    merged = {frozenset(m): j for j, m in enumerate(members) if len(m) > 1}
    # a merged single-member node cannot exist (>= 2 members), so the sets agree exactly
    assert set(merged) == set(ref)
    for ids, (K, com, pm, mid) in ref.items():
        j = merged[ids]
        assert int(res["mult"][j]) == K
        assert int(res["id"][j]) == mid
        assert int(res["type"][j]) == 1
        for d, key in enumerate(("x", "y", "z")):
            assert abs(res[key][j] - float(com[d])) <= 4e-16 * L
        pscale = max(abs(float(v)) for v in pm) + 1.0
        for d, key in enumerate(("px", "py", "pz")):
            assert abs(res[key][j] - float(pm[d])) <= 1e-14 * pscale
    # survivors are untouched
    for j, m in enumerate(members):
        if len(m) == 1 and res["id"][j] == m[0]:
            i = int(np.nonzero(ps.id == m[0])[0][0])
            if frozenset(m) not in ref:
                assert res["x"][j] == ps.x[i] and res["px"][j] == ps.px[i]
                assert res["mult"][j] == ps.mult[i] and res["type"][j] == ps.type[i]


def test_lattice_all_outside_reduces_to_lambda_over_lmax_cubed():
    """Every node outside: N_fin/N_init = (lambda/l_max)^3; the paper's printed bound for the
    fiducial l_max = 4 lambda is 0.0157, and Sec. 3.3 quotes mean mass ratios 8 (2 lambda) and
    64 (4 lambda)."""
    g = _golden("particle_reduction_bound.txt")
    n_side, L = 16, 16.0
    ps = dzs_ics.lattice(n_side, L)
    for j, mass_ratio in ((2, g["mass_ratio_lmax_2"]), (4, g["mass_ratio_lmax_4"])):
        k_min = oracle.k_min_for(n_side, j)
        assert L / 2 ** k_min == j * L / n_side
        res, group_of, nm = oracle.coarsen(ps, [0.0, 0.0, 0.0], 0.0, 0.0, 1e9, k_min)
        ratio = res["x"].shape[0] / ps.n
        assert ratio == (1.0 / j) ** 3
        assert np.all(res["mult"] == mass_ratio)
        if j == 4:
            # the paper prints four decimals: agree to its last printed digit
            assert abs(ratio - g["n_fin_over_n_init_lmax_4"]) <= 1e-4


def test_no_merge_when_lightcone_covers_box():
    L = 100.0
    ps = dzs_ics.clustered_random(5000, L, seed=7)
    R = math.sqrt(3) / 2 * L
    res, group_of, nm = oracle.coarsen(ps, [0.0, 0.0, 0.0], R, 0.0, 1e6, 1)
    assert nm == 0 and res["x"].shape[0] == ps.n
    # identity map: survivors keep their values
    order = np.argsort(res["id"])
    assert np.array_equal(res["x"][order], ps.x[np.argsort(ps.id)])


def test_config1_zeldovich_nodes_are_full_octets():
    """32^3 at z=49, l_max = 2 lambda: ZA displacements are far below lambda/2, so each level-4
    cube holds its 8 lattice particles and every merged node has exactly 8 members.  With
    theta = 1 nodes merge beyond R_lc + b + 2 lambda = 41.875 Mpc/h (min image), i.e. in ~69%
    of the box volume (1 - 4/3 pi 41.875^3 / 100^3)."""
    ps = dzs_ics.zeldovich(32, 100.0, 1.0 / 50.0, seed=20050528, spectrum="powerlaw")
    assert ps.max_disp < 100.0 / 32 / 2
    k_min = oracle.k_min_for(32, 2)
    assert k_min == 4
    res, group_of, nm = oracle.coarsen(ps, [0.0, 0.0, 0.0], 20.0, 5 * 100.0 / 32, 1.0, k_min)
    merged = res["type"] == 1
    assert np.all(res["mult"][merged] == 8)
    frac = 8 * merged.sum() / ps.n
    expected = 1 - 4 / 3 * math.pi * 41.875 ** 3 / 100.0 ** 3
    assert abs(frac - expected) < 0.03
    # theta = 0.1: threshold 20 + 15.625 + 62.5 > sqrt(3)/2 L -> nothing merges
    res2, _, nm2 = oracle.coarsen(ps, [0.0, 0.0, 0.0], 20.0, 5 * 100.0 / 32, 0.1, k_min)
    assert nm2 == 0


def test_conservation_and_order_independence():
    L = 50.0
    ps = dzs_ics.merged_state(dzs_ics.clustered_random(20000, L, seed=9, vel=500.0), seed=4)
    res, group_of, nm = oracle.coarsen(ps, [0.0, 0.0, 0.0], 5.0, 1.0, 0.7, 2)
    assert nm > 100
    assert int(res["mult"].astype(np.int64).sum()) == int(ps.mult.astype(np.int64).sum())
    m0 = ps.mult.astype(np.float64)
    m1 = res["mult"].astype(np.float64)
    for a, b in (("px", "px"), ("py", "py"), ("pz", "pz"), ("x", "x"), ("y", "y"), ("z", "z")):
        before = math.fsum(m0 * getattr(ps, a))
        after = math.fsum(m1 * res[b])
        scale = math.fsum(np.abs(m0 * getattr(ps, a)))
        assert abs(before - after) <= 1e-14 * scale
    # a shuffled copy gives the same result (canonical (key, id) summation order)
    perm = dzs_ics.rng(1).permutation(ps.n)
    ps2 = ps.take(perm)
    res2, group_of2, nm2 = oracle.coarsen(ps2, [0.0, 0.0, 0.0], 5.0, 1.0, 0.7, 2)
    o1, o2 = np.argsort(res["id"]), np.argsort(res2["id"])
    for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
        assert np.array_equal(res[k][o1], res2[k][o2])
    new_id1 = res["id"][group_of]
    new_id2 = res2["id"][group_of2]
    assert np.array_equal(new_id1[perm], new_id2)

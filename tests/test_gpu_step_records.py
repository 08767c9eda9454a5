"""GPU parity of whole steps that emit lightcone records while they coarsen.

* kdk_step on a mixed-mass 32^3 box late in the run (a 0.985 -> 0.99, the lightcone sphere
  sweeping through the box): lightcone selection by id, the records' multiplicities and
  momenta bit-exact, crossing times to 1e-12 on a sample, the coarsening (grouping, merged
  particles) and the drifted positions bit-exact, forces within the plain (1e-9) or
  precision (1e-5 of |g_PM| + |g_short|) bar, all against the FP64 oracle's step;
* the same step on the library's own kick, drift and lightcone factors (dzs_step_factors)
  against the oracle's step on its own factors: the two cosmologies agree to 1e-13, so the
  positions, momenta and forces agree to that level and the selection is identical;
* kdk_step_batch on boxes first coarsened by dzs_coarsen (checked bit-exact against the
  oracle's coarsening) to multiplicities up to 64, stepped while the sphere crosses some of
  them: per box, records by id, positions bit-exact, forces and momenta as above.
"""
import math
import sys

import numpy as np
import pytest

import dzs_ics
import oracle

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2005_05328_amd as dz
    return dz


def _rms(g, ref, scale=None):
    s2 = np.sum(ref ** 2, axis=0) if scale is None else scale ** 2
    return math.sqrt(np.mean(np.sum((g - ref) ** 2, axis=0)) / np.mean(s2))


def _parts(ps, obox, ng, r_s, r_cut):
    """|g_PM| + |g_short| per particle: the scale FP32 rounding is relative to."""
    gp = oracle.pm_force(ps.x, ps.y, ps.z, ps.mult, obox, ng, r_s)
    gs = oracle.short_range(ps.x, ps.y, ps.z, ps.mult, obox, r_s, r_cut)
    return np.sqrt((gp ** 2).sum(0)) + np.sqrt((gs ** 2).sum(0))


def _kicked(ps, g, K):
    return np.stack([oracle.kick(getattr(ps, k), g[a], K) for a, k in enumerate(("px", "py", "pz"))])


def _check_records(rec, ref_ids, ps0, p_kick, a0, a1, n_solve=20):
    """Records of one run against the oracle's selection: the same ids (each once), the
    multiplicity and the kicked momentum of each, and crossing times on a sample."""
    ids = np.asarray(rec["id"])
    assert ids.size == np.unique(ids).size
    assert np.array_equal(np.sort(ids), np.sort(ref_ids))
    where = {int(i): k for k, i in enumerate(ps0.id)}
    idx = np.array([where[int(i)] for i in ids], np.int64)
    assert np.array_equal(rec["mult"], ps0.mult[idx])
    assert np.array_equal(rec["p"], p_kick[:, idx].T)
    d0 = np.stack([oracle.min_image(getattr(ps0, k) - 0.0, ps0.L) for k in ("x", "y", "z")])
    for r in np.argsort(ids)[:: max(1, ids.size // n_solve)]:
        i = idx[r]
        p = p_kick[:, i]
        ac = oracle.crossing_time(d0[:, i], p, a0, a1)
        assert abs(rec["a_cross"][r] - ac) <= 1e-12, (rec["a_cross"][r], ac)
        dref = d0[:, i] + p * oracle.drift_factor(a0, ac) if ac > a0 else d0[:, i]
        assert np.abs(rec["d"][r] - dref).max() <= 1e-9 * max(1.0, np.linalg.norm(dref))


def _late_box(seed, n_side=32, L=100.0, a=0.985):
    ps = dzs_ics.zeldovich(n_side, L, a, seed=seed, spectrum="bbks")
    ps = dzs_ics.merged_state(ps, seed=seed + 1, frac=0.2, max_mult=8)
    ps.id = dzs_ics.rng(seed + 2).permutation(ps.n).astype(np.uint32)
    return ps


@pytest.mark.parametrize("fp32", [False, True])
def test_kdk_step_emits_records_while_it_coarsens(dz, fp32):
    import torch
    from test_gpu_parity import _fp32_force_error
    n_side, L, ng = 32, 100.0, 64
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    lam = L / n_side
    ps = _late_box(20050561)
    m0 = dzs_ics.particle_mass(L, n_side ** 3)
    box, obox = dz.make_box(L, m0, lam / 40), oracle.Box(L=L, m0=m0, eps0=lam / 40)
    a0, a1 = 0.985, 0.99
    fac = oracle.step_factors(a0, a1)
    fac.update(a0=a0, a1=a1)
    cp = dict(R_lc=math.sqrt(fac["chi2_1"]), b=5 * lam, theta=1.0, k_min=4)
    g0 = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, obox, ng, r_s, r_cut)
    ref, ref_g, rec_ref, cres = oracle.kdk_step(ps, g0, obox, fac, ng, r_s, r_cut,
                                                [0.0, 0.0, 0.0], coarsen_params=cp, solve=False)
    prec = dz.DZS_FP32 if fp32 else dz.DZS_FP64
    sp = dz.step_factors(a0, a1, 0.3)
    sp.K1, sp.K2 = fac["K1"], fac["K2"]
    sp.lc.D, sp.lc.chi2_0, sp.lc.chi2_1 = fac["D"], fac["chi2_0"], fac["chi2_1"]
    sp.do_lightcone, sp.do_coarsen = 1, 1
    sp.coarsen.R_lc, sp.coarsen.b = cp["R_lc"], cp["b"]
    sp.coarsen.theta, sp.coarsen.k_min = cp["theta"], cp["k_min"]
    sp.pm = dz.PMParams(ng, prec, r_s, 0, 0)
    sp.tree = dz.TreeParams(r_s, r_cut, 0.0, 8, 32, prec, 0)
    ctx = dz.Context(ps.n, ng)
    st = dz.State.from_host(ps, g=g0)
    ring = dz.LCRing(ps.n)
    ring.reset()
    rep = ctx.kdk_step(box, st, sp, ring)
    torch.cuda.synchronize()
    out = st.to_host()
    rec = ring.records()
    ctx.close()
    _log(f"kdk fp32={fp32}: {rec['count']} records, {rep.n_groups} merged nodes, "
         f"n {ps.n} -> {st.n}")
    assert rec["overflow"] == 0 and rec["count"] > 1000
    assert rep.n_groups == cres[2] > 100 and st.n == ref.n
    _check_records(rec, rec_ref["id"], ps, _kicked(ps, g0, fac["K1"]), a0, a1)
    o, r = np.argsort(out["id"]), np.argsort(ref.id)
    for k in ("x", "y", "z", "mult", "id", "type"):
        assert np.array_equal(out[k][o], getattr(ref, k)[r]), k
    g = np.stack([out["gx"][o], out["gy"][o], out["gz"][o]])
    rg = ref_g[:, r]
    if fp32:
        parts = _parts(ref, obox, ng, r_s, r_cut)[r]
        err, n_flip, bounded = _fp32_force_error(g, rg, ref.take(r), obox, r_s, r_cut, norm=parts)
        _log(f"  force rms / (|g_PM| + |g_short|) {err:.3e}, {n_flip} cutoff flips")
        assert bounded and err <= 1e-5
    else:
        err = _rms(g, rg)
        _log(f"  force rms rel {err:.3e}")
        assert err <= 1e-9
    for a, k in enumerate(("px", "py", "pz")):
        dp = out[k][o] - getattr(ref, k)[r] - fac["K2"] * (g[a] - rg[a])
        assert np.abs(dp).max() <= 1e-9 * np.abs(getattr(ref, k)).max()


def test_kdk_step_on_the_library_own_factors(dz):
    """No factor is borrowed from the oracle: dzs_step_factors supplies K1, K2, D, chi^2 and
    the Chebyshev series.  Each side then steps on its own cosmology (agreeing to 1e-13)."""
    import torch
    n_side, L, ng = 32, 100.0, 64
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    lam = L / n_side
    ps = _late_box(20050571)
    m0 = dzs_ics.particle_mass(L, n_side ** 3)
    box, obox = dz.make_box(L, m0, lam / 40), oracle.Box(L=L, m0=m0, eps0=lam / 40)
    a0, a1 = 0.985, 0.99
    fac = oracle.step_factors(a0, a1)
    fac.update(a0=a0, a1=a1)
    cp = dict(R_lc=math.sqrt(fac["chi2_1"]), b=5 * lam, theta=1.0, k_min=4)
    g0 = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, obox, ng, r_s, r_cut)
    ref, ref_g, rec_ref, cres = oracle.kdk_step(ps, g0, obox, fac, ng, r_s, r_cut,
                                                [0.0, 0.0, 0.0], coarsen_params=cp, solve=False)
    sp = dz.step_factors(a0, a1, 0.3)
    sp.do_lightcone, sp.do_coarsen = 1, 1
    sp.coarsen.R_lc = math.sqrt(sp.lc.chi2_1)
    sp.coarsen.b, sp.coarsen.theta, sp.coarsen.k_min = cp["b"], cp["theta"], cp["k_min"]
    sp.pm = dz.PMParams(ng, dz.DZS_FP64, r_s, 0, 0)
    sp.tree = dz.TreeParams(r_s, r_cut, 0.0, 8, 32, dz.DZS_FP64, 0)
    for mine, theirs in ((sp.K1, fac["K1"]), (sp.K2, fac["K2"]), (sp.lc.D, fac["D"]),
                         (sp.lc.chi2_0, fac["chi2_0"]), (sp.lc.chi2_1, fac["chi2_1"])):
        assert mine != 0.0 and abs(mine - theirs) <= 1e-13 * abs(theirs)
    ctx = dz.Context(ps.n, ng)
    st = dz.State.from_host(ps, g=g0)
    ring = dz.LCRing(ps.n)
    ring.reset()
    rep = ctx.kdk_step(box, st, sp, ring)
    torch.cuda.synchronize()
    out = st.to_host()
    rec = ring.records()
    ctx.close()
    _log(f"own factors: {rec['count']} records, {rep.n_groups} merged nodes")
    assert rec["count"] > 1000 and np.array_equal(np.sort(rec["id"]), np.sort(rec_ref["id"]))
    assert rep.n_groups == cres[2] > 100 and st.n == ref.n
    o, r = np.argsort(out["id"]), np.argsort(ref.id)
    for k in ("mult", "id", "type"):
        assert np.array_equal(out[k][o], getattr(ref, k)[r]), k
    for k in ("x", "y", "z"):
        d = out[k][o] - getattr(ref, k)[r]
        d -= L * np.round(d / L)
        assert np.abs(d).max() <= 1e-11 * L, k
    g = np.stack([out["gx"][o], out["gy"][o], out["gz"][o]])
    assert _rms(g, ref_g[:, r]) <= 1e-9
    for k in ("px", "py", "pz"):
        scale = np.abs(getattr(ref, k)).max()
        assert np.abs(out[k][o] - getattr(ref, k)[r]).max() <= 1e-9 * scale


# (particles per side, box side, mesh side, seed, DZS level): uneven counts, masses and meshes
BOXES = [(16, 50.0, 32, 401, 1), (24, 80.0, 48, 402, 2), (32, 120.0, 64, 403, 3),
         (12, 40.0, 24, 404, 1), (20, 70.0, 48, 405, 2)]


@pytest.mark.parametrize("fp32", [False, True])
def test_batched_step_of_coarsened_boxes_with_records(dz, fp32):
    import torch
    from test_gpu_parity import _fp32_force_error
    a0, a1 = 0.98, 0.985
    fac = oracle.step_factors(a0, a1)
    fac.update(a0=a0, a1=a1)
    prec = dz.DZS_FP32 if fp32 else dz.DZS_FP64
    cctx = dz.Context(32 ** 3 + 64, 64)
    sets, boxes, oboxes, first, ngs, rss, rcs, refs, g0s = [], [], [], [0], [], [], [], [], []
    id_base = 0
    for n_side, L, ng, seed, level in BOXES:
        lam = L / n_side
        ps = dzs_ics.zeldovich(n_side, L, a0, seed=seed, spectrum="bbks")
        ps.id = ps.id + np.uint32(id_base)
        id_base += ps.n
        m0 = dzs_ics.particle_mass(L, ps.n)
        box, obox = dz.make_box(L, m0, lam / 40), oracle.Box(L=L, m0=m0, eps0=lam / 40)
        k_min = oracle.k_min_for(n_side, 2 ** level)
        # coarsened once outside a prescribed sphere: the GPU's dzs_coarsen first, bit-exact
        # against the oracle's coarsening of the same box
        out_o, _, n_merged = oracle.coarsen(ps, [0.0, 0.0, 0.0], 0.25 * L, 0.0, 1.0, k_min)
        st = dz.State.from_host(ps)
        cp = dz.CoarsenParams()
        cp.R_lc, cp.b, cp.theta, cp.k_min = 0.25 * L, 0.0, 1.0, k_min
        rep = cctx.dzs_coarsen(box, st, cp)
        torch.cuda.synchronize()
        h = st.to_host()
        assert rep.n_groups == n_merged > 0 and st.n == out_o["x"].shape[0]
        o, r = np.argsort(h["id"]), np.argsort(out_o["id"])
        for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
            assert np.array_equal(h[k][o], out_o[k][r]), (seed, k)
        cps = dzs_ics.ParticleSet(*(out_o[k] for k in ("x", "y", "z", "px", "py", "pz", "mult",
                                                         "id", "type")), L=L)
        r_s = 1.25 * L / ng
        r_cut = 4.5 * r_s
        g0 = oracle.total_force(cps.x, cps.y, cps.z, cps.mult, obox, ng, r_s, r_cut)
        refs.append(oracle.kdk_step(cps, g0, obox, fac, ng, r_s, r_cut, [0.0, 0.0, 0.0],
                                    solve=False))
        sets.append(cps)
        g0s.append(g0)
        boxes.append(box)
        oboxes.append(obox)
        first.append(first[-1] + cps.n)
        ngs.append(ng)
        rss.append(r_s)
        rcs.append(r_cut)
    cctx.close()
    mults = np.concatenate([p.mult for p in sets])
    assert mults.max() >= 8

    class _P:
        pass
    allp = _P()
    for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
        setattr(allp, k, np.concatenate([getattr(p, k) for p in sets]))
    st = dz.State.from_host(allp, g=np.concatenate(g0s, axis=1))
    sp = dz.step_factors(a0, a1, 0.3)
    sp.K1, sp.K2 = fac["K1"], fac["K2"]
    sp.lc.D, sp.lc.chi2_0, sp.lc.chi2_1 = fac["D"], fac["chi2_0"], fac["chi2_1"]
    sp.do_lightcone, sp.do_coarsen = 1, 0
    sp.pm = dz.PMParams(0, prec, 0.0, 0, 0)
    sp.tree = dz.TreeParams(0.0, 0.0, 0.0, 8, 32, prec, 0)
    ring = dz.LCRing(first[-1])
    ring.reset()
    ctx = dz.Context(max_particles=first[-1] + 64, max_mesh_side=81)
    _log(f"coarsened batch: {first[-1]} particles in {len(BOXES)} boxes, fp32={fp32}")
    ctx.kdk_step_batch(boxes, first, ngs, rss, rcs, st, sp, ring)
    torch.cuda.synchronize()
    ctx.check()
    out = st.to_host()
    rec = ring.records()
    ctx.close()
    assert rec["overflow"] == 0
    with_records = 0
    for b, (ps, ob) in enumerate(zip(sets, oboxes)):
        lo, hi = first[b], first[b + 1]
        ref, ref_g, rec_ref, _ = refs[b]
        sel = (rec["id"] >= ps.id.min()) & (rec["id"] <= ps.id.max())
        rb = {k: v[sel] for k, v in rec.items() if isinstance(v, np.ndarray)}
        _check_records(rb, rec_ref["id"], ps, _kicked(ps, g0s[b], fac["K1"]), a0, a1, n_solve=8)
        with_records += rb["id"].size > 0
        o = np.argsort(out["id"][lo:hi]) + lo
        r = np.argsort(ref.id)
        assert np.array_equal(out["id"][o], ref.id[r])
        for k in ("x", "y", "z", "mult", "type"):
            assert np.array_equal(out[k][o], getattr(ref, k)[r]), (b, k)
        g = np.stack([out["gx"][o], out["gy"][o], out["gz"][o]])
        rg = ref_g[:, r]
        if fp32:
            parts = _parts(ref, ob, ngs[b], rss[b], rcs[b])[r]
            err, n_flip, bounded = _fp32_force_error(g, rg, ref.take(r), ob, rss[b], rcs[b],
                                                     norm=parts)
            assert bounded and err <= 1e-5, (b, err)
        else:
            err = _rms(g, rg)
            assert err <= 1e-9, (b, err)
        _log(f"  box {b}: n={hi - lo}, max mult {ps.mult.max()}, {rb['id'].size} records, "
             f"force err {err:.3e}")
        for a, k in enumerate(("px", "py", "pz")):
            dp = out[k][o] - getattr(ref, k)[r] - fac["K2"] * (g[a] - rg[a])
            assert np.abs(dp).max() <= 1e-9 * np.abs(getattr(ref, k)).max()
    assert with_records >= 2

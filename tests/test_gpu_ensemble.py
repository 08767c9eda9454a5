"""Run control of a batched ensemble (paper Sec. 4.1.1): five boxes in one state, each
coarsened in its own range by the library (bit-exact against the oracle's coarsening of that
box), the halt predicate deciding to re-pack as the count falls below the threshold, the
survivors re-packed into a state fitted to their count, and one batched step of the
re-packed ensemble against the oracle's step of each box alone."""
import math
import sys

import numpy as np
import pytest

import dzs_ics
import oracle

pytestmark = pytest.mark.gpu

BOXES = [(16, 50.0, 32, 501), (24, 80.0, 48, 502), (32, 120.0, 64, 503), (12, 40.0, 24, 504),
         (20, 70.0, 48, 505)]


def test_coarsen_repack_and_step_the_ensemble():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2005_05328_amd as dz
    from paper_2005_05328_amd import ensemble
    a0 = 0.5
    sets, boxes, oboxes, first, ngs, rss, rcs, cps = [], [], [], [0], [], [], [], []
    id_base = 0
    for n_side, L, ng, seed in BOXES:
        ps = dzs_ics.zeldovich(n_side, L, a0, seed=seed, spectrum="bbks")
        ps.id = ps.id + np.uint32(id_base)
        id_base += ps.n
        lam = L / n_side
        m0 = dzs_ics.particle_mass(L, ps.n)
        boxes.append(dz.make_box(L, m0, lam / 40))
        oboxes.append(oracle.Box(L=L, m0=m0, eps0=lam / 40))
        sets.append(ps)
        first.append(first[-1] + ps.n)
        ngs.append(ng)
        rss.append(1.25 * L / ng)
        rcs.append(4.5 * 1.25 * L / ng)
        cp = dz.CoarsenParams()
        cp.R_lc, cp.b, cp.theta = 0.3 * L, 0.0, 1.0
        cp.k_min = oracle.k_min_for(n_side, 2)
        cps.append(cp)

    class _P:
        pass
    allp = _P()
    for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
        setattr(allp, k, np.concatenate([getattr(p, k) for p in sets]))
    N = first[-1]
    st = dz.State.from_host(allp)
    cctx = dz.Context(max(p.n for p in sets) + 64, max(ngs))
    counts, reports = ensemble.coarsen_boxes(cctx, boxes, st, first, cps)
    torch.cuda.synchronize()
    cctx.close()
    ratio, reasons = ensemble.control(counts, N, min_ratio=0.9)
    print(f"ensemble: {N} -> {sum(counts)} particles (R = {ratio:.3f}), reasons {reasons}",
          flush=True)
    assert reasons & dz._abi.DZS_HALT_RATIO
    packed, first2 = ensemble.repack(st, first, counts)
    assert packed.capacity == sum(counts) == first2[-1] and packed.n == first2[-1]
    h = packed.to_host()
    # each box's survivors: the oracle's coarsening of that box, bit for bit
    refs = []
    fac = oracle.step_factors(a0, a0 * 1.02)
    fac.update(a0=a0, a1=a0 * 1.02)
    for b, (ps, cp) in enumerate(zip(sets, cps)):
        out, _, nm = oracle.coarsen(ps, [0.0, 0.0, 0.0], cp.R_lc, cp.b, cp.theta, cp.k_min)
        assert reports[b].n_groups == nm > 0 and counts[b] == out["x"].shape[0]
        lo, hi = first2[b], first2[b + 1]
        o, r = np.argsort(h["id"][lo:hi]) + lo, np.argsort(out["id"])
        for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
            assert np.array_equal(h[k][o], out[k][r]), (b, k)
        cps_ = dzs_ics.ParticleSet(*(out[k] for k in ("x", "y", "z", "px", "py", "pz", "mult",
                                                       "id", "type")), L=ps.L)
        g0 = oracle.total_force(cps_.x, cps_.y, cps_.z, cps_.mult, oboxes[b], ngs[b], rss[b],
                                rcs[b])
        ref, ref_g, _, _ = oracle.kdk_step(cps_, g0, oboxes[b], fac, ngs[b], rss[b], rcs[b],
                                           [0.0, 0.0, 0.0], solve=False)
        # the step's input force in the packed order
        ro = np.argsort(cps_.id)
        pos = np.searchsorted(cps_.id[ro], h["id"][lo:hi])
        for a, k in enumerate(("gx", "gy", "gz")):
            getattr(packed, k)[lo:hi] = torch.from_numpy(g0[a][ro][pos]).cuda()
        refs.append((ref, ref_g))
    # one batched step of the re-packed ensemble, in a context fitted to it
    sp = dz.step_factors(a0, a0 * 1.02, 0.3)
    sp.K1, sp.K2 = fac["K1"], fac["K2"]
    sp.lc.D, sp.lc.chi2_0, sp.lc.chi2_1 = fac["D"], fac["chi2_0"], fac["chi2_1"]
    sp.do_lightcone, sp.do_coarsen = 0, 0
    sp.pm = dz.PMParams(0, dz.DZS_FP64, 0.0, 0, 0)
    sp.tree = dz.TreeParams(0.0, 0.0, 0.0, 8, 32, dz.DZS_FP64, 0)
    ctx = dz.Context(first2[-1] + 64, 81)
    ctx.kdk_step_batch(boxes, first2, ngs, rss, rcs, packed, sp)
    torch.cuda.synchronize()
    ctx.check()
    out = packed.to_host()
    ctx.close()
    for b in range(len(BOXES)):
        lo, hi = first2[b], first2[b + 1]
        ref, ref_g = refs[b]
        o, r = np.argsort(out["id"][lo:hi]) + lo, np.argsort(ref.id)
        assert np.array_equal(out["id"][o], ref.id[r])
        for k in ("x", "y", "z", "mult"):
            assert np.array_equal(out[k][o], getattr(ref, k)[r]), (b, k)
        g = np.stack([out["gx"][o], out["gy"][o], out["gz"][o]])
        rg = ref_g[:, r]
        err = math.sqrt(((g - rg) ** 2).sum(0).mean() / (rg ** 2).sum(0).mean())
        print(f"  box {b}: {hi - lo} particles, force rms rel {err:.2e}", flush=True)
        assert err <= 1e-9

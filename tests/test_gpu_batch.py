"""GPU parity of the batched step: several independent boxes of different sizes, masses and
meshes advanced by one kdk_step_batch call, each box against the FP64 oracle's step of that
box alone.  Bars: drifted positions bit-exact (the drift is the same FP64 arithmetic per
box); forces at opening angle 0 within rms 1e-9 (plain form) of the oracle's direct sum +
PM; momenta within 1e-9 of their scale; the precision form within the 1e-5 force bar."""
import math
import sys

import numpy as np
import pytest

import dzs_ics
import oracle

pytestmark = pytest.mark.gpu

# (particles per side, box side, mesh side, seed): uneven counts, masses and meshes
BOXES = [(16, 50.0, 32, 301), (24, 80.0, 48, 302), (32, 120.0, 64, 303), (12, 40.0, 24, 304),
         (20, 70.0, 48, 305)]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2005_05328_amd as dz
    return dz


def _setup(dz):
    sets, boxes, oboxes, first, ng, r_s, r_cut = [], [], [], [0], [], [], []
    id_base = 0
    for n_side, L, g, seed in BOXES:
        ps = dzs_ics.zeldovich(n_side, L, 0.02, seed=seed, spectrum="bbks")
        ps.id = ps.id + np.uint32(id_base)
        id_base += ps.n
        lam = L / n_side
        m0 = dzs_ics.particle_mass(L, ps.n)
        boxes.append(dz.make_box(L, m0, lam / 40))
        oboxes.append(oracle.Box(L=L, m0=m0, eps0=lam / 40))
        sets.append(ps)
        first.append(first[-1] + ps.n)
        ng.append(g)
        r_s.append(1.25 * L / g)
        r_cut.append(4.5 * 1.25 * L / g)
    return sets, boxes, oboxes, first, ng, r_s, r_cut


def _concat(sets):
    class _P:
        pass
    out = _P()
    for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
        setattr(out, k, np.concatenate([getattr(p, k) for p in sets]))
    return out


@pytest.mark.parametrize("fp32", [False, True])
def test_batched_step_matches_the_oracle_per_box(dz, fp32):
    import torch
    sets, boxes, oboxes, first, ng, r_s, r_cut = _setup(dz)
    prec = dz.DZS_FP32 if fp32 else dz.DZS_FP64
    a0, a1 = 0.02, 0.02 * math.exp(0.07824)
    fac = oracle.step_factors(a0, a1)
    fac.update(a0=a0, a1=a1)
    g0s, refs = [], []
    for ps, ob, g, rs, rc in zip(sets, oboxes, ng, r_s, r_cut):
        g0 = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, ob, g, rs, rc)
        ref, ref_g, _, _ = oracle.kdk_step(ps, g0, ob, fac, g, rs, rc, [0.0, 0.0, 0.0],
                                           solve=False)
        g0s.append(g0)
        refs.append((ref, ref_g))
    allp = _concat(sets)
    st = dz.State.from_host(allp, g=np.concatenate(g0s, axis=1))
    sp = dz.step_factors(a0, a1, 0.3)
    sp.K1, sp.K2 = fac["K1"], fac["K2"]
    sp.lc.D, sp.lc.chi2_0, sp.lc.chi2_1 = fac["D"], fac["chi2_0"], fac["chi2_1"]
    sp.do_lightcone, sp.do_coarsen = 1, 0
    sp.pm = dz.PMParams(0, prec, 0.0, 0, 0)
    sp.tree = dz.TreeParams(0.0, 0.0, 0.0, 8, 32, prec, 0)
    ring = dz.LCRing(1000)
    ring.reset()
    ctx = dz.Context(max_particles=first[-1] + 64, max_mesh_side=81)
    _log(f"batch of {len(BOXES)} boxes, {first[-1]} particles, fp32={fp32}")
    ctx.kdk_step_batch(boxes, first, ng, r_s, r_cut, st, sp, ring)
    torch.cuda.synchronize()
    out = st.to_host()
    ctx.close()
    assert ring.records()["count"] == 0          # chi(z = 49) >> L
    for b, (ps, ob) in enumerate(zip(sets, oboxes)):
        lo, hi = first[b], first[b + 1]
        ref, ref_g = refs[b]
        o = np.argsort(out["id"][lo:hi]) + lo
        r = np.argsort(ref.id)
        # each box keeps its own particles in its own range
        assert np.array_equal(out["id"][o], ref.id[r])
        for k in ("x", "y", "z", "mult", "type"):
            assert np.array_equal(out[k][o], getattr(ref, k)[r]), (b, k)
        g = np.stack([out["gx"][o], out["gy"][o], out["gz"][o]])
        rg = ref_g[:, r]
        err = math.sqrt(((g - rg) ** 2).sum(0).mean() / (rg ** 2).sum(0).mean())
        # the force of a z = 49 lattice is a small residual: scale by the parts' magnitude
        gp = oracle.pm_force(ref.x, ref.y, ref.z, ref.mult, ob, ng[b], r_s[b])[:, r]
        gs = oracle.short_range(ref.x, ref.y, ref.z, ref.mult, ob, r_s[b], r_cut[b])[:, r]
        parts = np.sqrt((gp ** 2).sum(0)) + np.sqrt((gs ** 2).sum(0))
        err_p = math.sqrt(((g - rg) ** 2).sum(0).mean() / (parts ** 2).mean())
        _log(f"  box {b}: n={hi - lo} force rms rel {err:.3e}, of the parts {err_p:.3e}")
        if fp32:
            assert err_p <= 1e-5
        else:
            assert err <= 1e-9
        for a, k in enumerate(("px", "py", "pz")):
            dp = out[k][o] - getattr(ref, k)[r] - fac["K2"] * (g[a] - rg[a])
            assert np.abs(dp).max() <= 1e-9 * np.abs(getattr(ref, k)).max()


def test_batched_step_rejects_bad_batches(dz):
    sets, boxes, _, first, ng, r_s, r_cut = _setup(dz)
    st = dz.State.from_host(_concat(sets))
    sp = dz.step_factors(0.5, 0.51, 0.3)
    sp.do_lightcone, sp.do_coarsen = 0, 0
    sp.pm = dz.PMParams(0, dz.DZS_FP64, 0.0, 0, 0)
    sp.tree = dz.TreeParams(0.0, 0.0, 0.5, 8, 32, dz.DZS_FP64, 0)
    ctx = dz.Context(max_particles=first[-1] + 64, max_mesh_side=81)
    bad_first = list(first)
    bad_first[-1] -= 1
    with pytest.raises(dz.DZSError):
        ctx.kdk_step_batch(boxes, bad_first, ng, r_s, r_cut, st, sp)
    bad_rc = list(r_cut)
    bad_rc[1] *= 1.1                               # a different r_cut / r_s
    with pytest.raises(dz.DZSError):
        ctx.kdk_step_batch(boxes, first, ng, r_s, bad_rc, st, sp)
    bad_ng = list(ng)
    bad_ng[0] = 35                                 # not 2^a 3^b
    with pytest.raises(dz.DZSError):
        ctx.kdk_step_batch(boxes, first, bad_ng, r_s, r_cut, st, sp)
    big = dz.Context(max_particles=first[-1] + 64, max_mesh_side=36)
    with pytest.raises(dz.DZSError):               # meshes exceed the context
        big.kdk_step_batch(boxes, first, ng, r_s, r_cut, st, sp)
    sp.do_coarsen = 1
    with pytest.raises(dz.DZSError):
        ctx.kdk_step_batch(boxes, first, ng, r_s, r_cut, st, sp)
    ctx.close()
    big.close()


def test_captured_batched_step_replays_match_eager_steps(dz):
    """kdk_step_batch captured once into a HIP graph (torch.cuda.graph) and replayed for four
    consecutive steps, each with its own factors staged by kdk_step_batch_stage, against the
    same four steps called eagerly on a second context: positions, momenta, forces, ids and
    the lightcone records agree bit for bit after every replay (the step is deterministic)."""
    import torch
    sets, boxes, _, first, ng, r_s, r_cut = _setup(dz)
    allp = _concat(sets)
    a = np.exp(np.linspace(math.log(0.96), 0.0, 5))   # late: the lightcone passes the boxes
    steps = []
    for s in range(4):
        sp = dz.step_factors(float(a[s]), float(a[s + 1]), 0.3)
        sp.do_lightcone, sp.do_coarsen = 1, 0
        sp.pm = dz.PMParams(0, dz.DZS_FP32, 0.0, 0, 0)
        sp.tree = dz.TreeParams(0.0, 0.0, 0.5, 16, 32, dz.DZS_FP32, 0)
        steps.append(sp)
    st_e = dz.State.from_host(allp)
    st_g = dz.State.from_host(allp)
    st_w = dz.State.from_host(allp)
    ring_e, ring_g, ring_w = dz.LCRing(first[-1]), dz.LCRing(first[-1]), dz.LCRing(first[-1])
    for r in (ring_e, ring_g, ring_w):
        r.reset()
    ctx_e = dz.Context(max_particles=first[-1] + 64, max_mesh_side=81)
    ctx_g = dz.Context(max_particles=first[-1] + 64, max_mesh_side=81)
    # one eager call prepares the graph context's tables (this synchronises, so not captured)
    ctx_g.kdk_step_batch(boxes, first, ng, r_s, r_cut, st_w, steps[0], ring_w)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ctx_g.kdk_step_batch(boxes, first, ng, r_s, r_cut, st_g, steps[0], ring_g)
    torch.cuda.synchronize()
    for s in range(4):
        ctx_g.kdk_step_batch_stage(steps[s])
        graph.replay()
        torch.cuda.synchronize()
        ctx_e.kdk_step_batch(boxes, first, ng, r_s, r_cut, st_e, steps[s], ring_e)
        torch.cuda.synchronize()
        he, hg = st_e.to_host(), st_g.to_host()
        for k in ("x", "y", "z", "px", "py", "pz", "gx", "gy", "gz", "id", "mult"):
            assert np.array_equal(he[k], hg[k]), (s, k)
        re, rg = ring_e.records(), ring_g.records()
        _log(f"replay {s}: {rg['count']} lightcone records")
        assert re["count"] == rg["count"]
        oe, og = np.argsort(re["id"]), np.argsort(rg["id"])
        assert np.array_equal(re["id"][oe], rg["id"][og])
        assert np.array_equal(re["a_cross"][oe], rg["a_cross"][og])
    assert ring_g.records()["count"] > 0
    ctx_g.check()
    ctx_e.check()
    ctx_e.close()
    ctx_g.close()


def test_batched_steps_back_to_back_are_deterministic(dz):
    """Ten batched steps enqueued back to back (no synchronisation between calls) twice from
    the same state give bit-identical states: each call's factors travel with its own kernels
    (a shared host staging buffer overwritten by the next call before its copy ran once made
    steps use their successor's factors)."""
    import torch
    sets, boxes, _, first, ng, r_s, r_cut = _setup(dz)
    allp = _concat(sets)
    a = np.exp(np.linspace(math.log(0.1), math.log(0.1) + 0.5, 11))
    ctx = dz.Context(max_particles=first[-1] + 64, max_mesh_side=81)
    ring = dz.LCRing(1024)
    outs = []
    for rep in range(2):
        st = dz.State.from_host(allp)
        ring.reset()
        torch.cuda.synchronize()
        for s in range(10):
            sp = dz.step_factors(float(a[s]), float(a[s + 1]), 0.3)
            sp.do_lightcone, sp.do_coarsen = 1, 0
            sp.pm = dz.PMParams(0, dz.DZS_FP64, 0.0, 0, 0)
            sp.tree = dz.TreeParams(0.0, 0.0, 0.5, 32, 64, dz.DZS_FP64, 0)
            ctx.kdk_step_batch(boxes, first, ng, r_s, r_cut, st, sp, ring)
        torch.cuda.synchronize()
        outs.append(st.to_host())
    ctx.check()
    ctx.close()
    for k in ("x", "y", "z", "px", "py", "pz", "gx", "gy", "gz", "id"):
        assert np.array_equal(outs[0][k], outs[1][k]), k


@pytest.mark.parametrize("coarse_meshes", [False, True])
def test_batched_pm_tiles_give_identical_steps(dz, coarse_meshes):
    """The LDS tiles of deposit and interpolation in a batch (a chunk spanning two boxes reads
    and adds directly): one batched step without tiles, with tiles of 256 and with the default
    gives bit-identical states.  With meshes of about one point per particle the
    interpolation uses its tiles too."""
    import torch
    sets, boxes, _, first, ng, r_s, r_cut = _setup(dz)
    if coarse_meshes:
        ng = [16, 24, 32, 12, 18]
        r_s = [1.25 * b.L / g for b, g in zip(boxes, ng)]
        r_cut = [4.5 * r for r in r_s]
        assert 2 * first[-1] >= sum(g ** 3 for g in ng)
    allp = _concat(sets)
    ctx = dz.Context(max_particles=first[-1] + 64, max_mesh_side=81)
    ring = dz.LCRing(1024)
    outs = []
    for chunk in (-1, 256, 0):
        st = dz.State.from_host(allp)
        ring.reset()
        sp = dz.step_factors(0.1, 0.11, 0.3)
        sp.do_lightcone, sp.do_coarsen = 1, 0
        sp.pm = dz.PMParams(0, dz.DZS_FP64, 0.0, 0, chunk)
        sp.tree = dz.TreeParams(0.0, 0.0, 0.5, 16, 32, dz.DZS_FP64, 0)
        _log(f"batched step, PM tile chunk {chunk}")
        ctx.kdk_step_batch(boxes, first, ng, r_s, r_cut, st, sp, ring)
        torch.cuda.synchronize()
        outs.append(st.to_host())
    ctx.check()
    ctx.close()
    for o in outs[1:]:
        for k in ("x", "y", "z", "px", "py", "pz", "gx", "gy", "gz", "id"):
            assert np.array_equal(outs[0][k], o[k]), k

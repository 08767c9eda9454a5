"""GPU checks of the C ABI's boundary contract: the target subset of tree_force, the presorted
form and its device-side order check, contexts without sorted copies, the box capacity of a
batch, and a kdk_step that only enqueues work (so it can be captured into a HIP graph and
replayed bit for bit)."""
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


def _case(n=20000, L=100.0, seed=71):
    ps = dzs_ics.merged_state(dzs_ics.clustered_random(n, L, seed=seed, r_clump=L / 50),
                              seed=seed + 1, max_mult=16)
    m0 = dzs_ics.particle_mass(L, n)
    return ps, m0


def _g(st):
    return np.stack([st.gx[: st.n].cpu().numpy(), st.gy[: st.n].cpu().numpy(),
                     st.gz[: st.n].cpu().numpy()])


@pytest.mark.parametrize("fp32", [False, True])
def test_tree_force_targets_equal_the_full_force_and_leave_the_rest(dz, fp32):
    """The force of a target subset is the same bits as that target's force in a call for
    every particle; entries of g outside the subset keep what they held."""
    import torch
    L, ng = 100.0, 64
    ps, m0 = _case()
    r_s = 1.25 * L / ng
    box = dz.make_box(L, m0, L / 27 / 40)
    prec = dz.DZS_FP32 if fp32 else dz.DZS_FP64
    tp = dz.TreeParams(r_s, 4.5 * r_s, 0.5, 8, 32, prec, 0)
    ctx = dz.Context(ps.n, ng)
    st = dz.State.from_host(ps)
    ctx.tree_force(box, st, tp)
    ctx.check()
    g_all = _g(st)
    t = np.sort(dzs_ics.rng(5).choice(ps.n, 777, replace=False)).astype(np.int32)
    for k in ("gx", "gy", "gz"):
        getattr(st, k).fill_(12345.0)
    tt = torch.from_numpy(t).cuda()
    ctx.tree_force(box, st, tp, targets=tt)
    ctx.check()
    g_sub = _g(st)
    assert np.array_equal(g_sub[:, t], g_all[:, t])
    rest = np.setdiff1d(np.arange(ps.n), t)
    assert np.all(g_sub[:, rest] == 12345.0)
    # accumulate adds to the targets only
    tp.accumulate = 1
    ctx.tree_force(box, st, tp, targets=tt)
    ctx.check()
    g_acc = _g(st)
    assert np.array_equal(g_acc[:, t], g_all[:, t] + g_all[:, t])
    assert np.all(g_acc[:, rest] == 12345.0)
    # an empty subset computes nothing
    ctx.tree_force(box, st, tp, targets=tt[:0])
    ctx.check()
    assert np.array_equal(_g(st), g_acc)
    ctx.close()


def test_tree_force_targets_match_the_oracle(dz):
    """A subset's force against the oracle's direct sum over every source (opening angle 0)."""
    L, ng = 100.0, 64
    ps, m0 = _case(n=12000, seed=73)
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    eps0 = L / 27 / 40
    box, obox = dz.make_box(L, m0, eps0), oracle.Box(L=L, m0=m0, eps0=eps0)
    import torch
    t = np.sort(dzs_ics.rng(9).choice(ps.n, 500, replace=False)).astype(np.int32)
    ref = oracle.short_range(ps.x, ps.y, ps.z, ps.mult, obox, r_s, r_cut, targets=t)
    ctx = dz.Context(ps.n, ng)
    st = dz.State.from_host(ps)
    ctx.tree_force(box, st, dz.TreeParams(r_s, r_cut, 0.0, 8, 32, dz.DZS_FP64, 0),
                   targets=torch.from_numpy(t).cuda())
    ctx.check()
    g = _g(st)[:, t]
    ctx.close()
    err = math.sqrt(np.mean(((g - ref) ** 2).sum(0)) / np.mean((ref ** 2).sum(0)))
    _log(f"target subset vs oracle: rms rel {err:.3e}")
    assert err <= 1e-10


def test_presorted_tree_force_and_its_order_check(dz):
    """On a state in key order, presorted = 1 gives the bits of the sorted-copy path; on a
    state out of order it computes nothing and dzs_check reports DZS_EINVAL, as it does for a
    target index out of range.  The next call is unaffected."""
    import torch
    L, ng = 100.0, 64
    ps, m0 = _case(seed=75)
    r_s = 1.25 * L / ng
    box = dz.make_box(L, m0, L / 27 / 40)
    ctx = dz.Context(ps.n, ng)
    st = dz.State.from_host(ps)
    ctx.sort_state(box, st)
    tp = dz.TreeParams(r_s, 4.5 * r_s, 0.5, 8, 32, dz.DZS_FP64, 0)
    ctx.tree_force(box, st, tp)
    ctx.check()
    g_copy = _g(st)
    tp.presorted = 1
    for k in ("gx", "gy", "gz"):
        getattr(st, k).zero_()
    ctx.tree_force(box, st, tp)
    ctx.check()
    assert np.array_equal(_g(st), g_copy)
    # out of order: reverse the state
    rev = dz.State.from_host(dzs_ics.ParticleSet(*(getattr(st, k)[: st.n].flip(0).cpu().numpy()
                                                   for k in ("x", "y", "z", "px", "py", "pz")),
                                                 st.mult[: st.n].flip(0).cpu().numpy().view(np.uint32),
                                                 st.id[: st.n].flip(0).cpu().numpy().view(np.uint32),
                                                 st.type[: st.n].flip(0).cpu().numpy(), L))
    for k in ("gx", "gy", "gz"):
        getattr(rev, k).fill_(7.0)
    ctx.tree_force(box, rev, tp)
    with pytest.raises(dz.DZSError, match="out of key order"):
        ctx.check()
    assert np.all(_g(rev) == 7.0)
    # a target index past n
    tp.presorted = 0
    bad = torch.tensor([0, ps.n + 5], dtype=torch.int32, device="cuda")
    ctx.tree_force(box, st, tp, targets=bad)
    with pytest.raises(dz.DZSError):
        ctx.check()
    # the context is usable afterwards
    ctx.tree_force(box, st, tp)
    ctx.check()
    assert np.array_equal(_g(st), g_copy)
    ctx.close()


def test_context_without_copies(dz):
    """DZS_CAP_NO_COPIES: tree_force needs presorted particles (DZS_EINVAL otherwise) and then
    gives the same force as a context with copies."""
    L, ng = 100.0, 64
    ps, m0 = _case(seed=77)
    r_s = 1.25 * L / ng
    box = dz.make_box(L, m0, L / 27 / 40)
    full = dz.Context(ps.n, ng)
    lean = dz.Context(ps.n, ng, no_copies=True)
    st = dz.State.from_host(ps)
    full.sort_state(box, st)
    tp = dz.TreeParams(r_s, 4.5 * r_s, 0.5, 8, 32, dz.DZS_FP32, 0)
    full.tree_force(box, st, tp)
    full.check()
    g_ref = _g(st)
    with pytest.raises(dz.DZSError, match="presorted"):
        lean.tree_force(box, st, tp)
    tp.presorted = 1
    lean.tree_force(box, st, tp)
    lean.check()
    assert np.array_equal(_g(st), g_ref)
    full.close()
    lean.close()


def test_batch_respects_the_box_capacity(dz):
    L, n_side, ng = 50.0, 12, 24
    sets = [dzs_ics.zeldovich(n_side, L, 0.1, seed=90 + b, spectrum="bbks") for b in range(3)]
    for b, p in enumerate(sets):
        p.id = p.id + np.uint32(b * p.n)

    class _P:
        pass
    allp = _P()
    for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
        setattr(allp, k, np.concatenate([getattr(p, k) for p in sets]))
    n = sum(p.n for p in sets)
    m0 = dzs_ics.particle_mass(L, n_side ** 3)
    boxes = [dz.make_box(L, m0, L / n_side / 40)] * 3
    first = [0, n_side ** 3, 2 * n_side ** 3, n]
    sp = dz.step_factors(0.1, 0.11, 0.3)
    sp.do_lightcone, sp.do_coarsen = 0, 0
    sp.pm = dz.PMParams(0, dz.DZS_FP64, 0.0, 0, 0)
    sp.tree = dz.TreeParams(0.0, 0.0, 0.5, 8, 32, dz.DZS_FP64, 0)
    rs = [1.25 * L / ng] * 3
    rc = [4.5 * r for r in rs]
    st = dz.State.from_host(allp)
    two = dz.Context(n + 64, 48, max_boxes=2)
    with pytest.raises(dz.DZSError, match="boxes exceed"):
        two.kdk_step_batch(boxes, first, [ng] * 3, rs, rc, st, sp)
    three = dz.Context(n + 64, 48, max_boxes=3)
    three.kdk_step_batch(boxes, first, [ng] * 3, rs, rc, st, sp)
    three.check()
    two.close()
    three.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_captured_kdk_step_replays_match_eager_steps(dz, fp32):
    """A kdk_step that cannot merge (coarsening on, but R_lc + b above the box's half
    diagonal) only enqueues work: captured once into a HIP graph and replayed four times it
    gives, after every replay, the bits of the same step called eagerly on a copy, lightcone
    records included."""
    import torch
    n_side, L, ng = 32, 100.0, 64
    ps = dzs_ics.zeldovich(n_side, L, 0.96, seed=20050581, spectrum="bbks")
    m0 = dzs_ics.particle_mass(L, ps.n)
    box = dz.make_box(L, m0, L / n_side / 40)
    prec = dz.DZS_FP32 if fp32 else dz.DZS_FP64
    r_s = 1.25 * L / ng
    a0, a1 = 0.97, 0.975
    sp = dz.step_factors(a0, a1, 0.3)
    sp.do_lightcone, sp.do_coarsen = 1, 1
    sp.coarsen.R_lc, sp.coarsen.b, sp.coarsen.theta, sp.coarsen.k_min = 0.9 * L, 5.0, 0.1, 4
    sp.pm = dz.PMParams(ng, prec, r_s, 0, 0)
    sp.tree = dz.TreeParams(r_s, 4.5 * r_s, 0.5, 8, 32, prec, 0)
    ctx_e, ctx_g = dz.Context(ps.n, ng), dz.Context(ps.n, ng)
    st_e, st_g = dz.State.from_host(ps), dz.State.from_host(ps)
    ring_e, ring_g = dz.LCRing(ps.n), dz.LCRing(ps.n)
    warm = dz.State.from_host(ps)
    ring_w = dz.LCRing(ps.n)
    ring_w.reset()
    ctx_g.kdk_step(box, warm, sp, ring_w)   # uploads the mesh tables (synchronises)
    torch.cuda.synchronize()
    ring_e.reset()
    ring_g.reset()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    with torch.cuda.graph(graph, stream=stream):
        ctx_g.kdk_step(box, st_g, sp, ring_g)
    torch.cuda.synchronize()
    seen = 0
    for r in range(4):
        ring_e.reset()
        ring_g.reset()
        graph.replay()
        torch.cuda.synchronize()
        ctx_e.kdk_step(box, st_e, sp, ring_e)
        torch.cuda.synchronize()
        he, hg = st_e.to_host(), st_g.to_host()
        for k in ("x", "y", "z", "px", "py", "pz", "gx", "gy", "gz", "id", "mult"):
            assert np.array_equal(he[k], hg[k]), (r, k)
        re_, rg = ring_e.records(), ring_g.records()
        _log(f"replay {r}: {rg['count']} records")
        assert re_["count"] == rg["count"]
        oe, og = np.argsort(re_["id"]), np.argsort(rg["id"])
        assert np.array_equal(re_["id"][oe], rg["id"][og])
        assert np.array_equal(re_["a_cross"][oe], rg["a_cross"][og])
        assert np.array_equal(re_["d"][oe], rg["d"][og])
        seen += rg["count"]
    assert seen > 0
    ctx_e.check()
    ctx_g.check()
    ctx_e.close()
    ctx_g.close()

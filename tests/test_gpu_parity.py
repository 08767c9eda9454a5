"""GPU parity: every call of the C ABI against the FP64 oracle on the same seeded inputs.

Bars (stated per test): bit-exact for Morton keys, the sort permutation, DZS grouping and the
merged particles, lightcone selection and the drifted positions; crossing times to 1e-12;
forces within an rms relative error (the plain FP64 form: 1e-10 at opening angle 0 where the
tree is the direct sum; <= 5e-3 at the production angle; PM 1e-8, set by the 2^-32
fixed-point deposit).
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


@pytest.fixture(scope="module")
def ctx(dz):
    c = dz.Context(max_particles=70000, max_mesh_side=64)
    yield c
    c.close()


def _box(dz, L, n_init, n_side=None):
    lam = L / (n_side if n_side else round(n_init ** (1 / 3)))
    m0 = dzs_ics.particle_mass(L, n_init)
    return dz.make_box(L, m0, lam / 40), oracle.Box(L=L, m0=m0, eps0=lam / 40)


def _rms_rel(g, ref):
    return math.sqrt(np.mean(np.sum((g - ref) ** 2, axis=0)) / np.mean(np.sum(ref ** 2, axis=0)))


def _fp32_force_error(g, ref, ps, box_o, r_s, r_cut, norm=None):
    """Error of a precision-form force, with the hard cutoff taken into account.

    A pair whose separation is within FP32 rounding of r_cut (relative 1e-7; 1e-6 is used) may
    be kept on one side and dropped on the other: that changes the target's force by
    G m_j S(r_cut / r_s) / r_cut^2 (S(4.5) = 1.8%: the cutoff is a jump).  Returns the rms
    relative error over the targets with no such pair, the number of targets with one, and
    whether every target is within its flips plus ten times the 1e-5 bar.  `norm` (per target) replaces |ref| as the scale."""
    from scipy.spatial import cKDTree
    L = box_o.L
    pos = np.stack([ps.x, ps.y, ps.z], axis=1) % L
    tree = cKDTree(pos, boxsize=L)
    pairs = tree.query_pairs(r_cut * (1 + 1e-6), output_type="ndarray")
    d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
    d -= L * np.round(d / L)
    near = pairs[np.sqrt((d ** 2).sum(1)) >= r_cut * (1 - 1e-6)]
    u = r_cut / r_s
    s_cut = math.erfc(u / 2) + u / math.sqrt(math.pi) * math.exp(-u * u / 4)
    jump = box_o.G * box_o.m0 * s_cut / r_cut ** 2
    flip = np.zeros(ps.n)
    np.add.at(flip, near[:, 0], jump * ps.mult[near[:, 1]])
    np.add.at(flip, near[:, 1], jump * ps.mult[near[:, 0]])
    err = np.sqrt(((g - ref) ** 2).sum(0))
    scale2 = (ref ** 2).sum(0) if norm is None else norm ** 2
    clean = flip == 0
    rms = math.sqrt(np.mean(err[clean] ** 2) / np.mean(scale2[clean]))
    bound = flip + 1e-5 * math.sqrt(np.mean(scale2)) * 10
    return rms, int((~clean).sum()), bool(np.all(err <= bound * 1.01))


# ------------------------------------------------------------------------------ keys, sort

@pytest.mark.parametrize("case", ["uniform", "clustered", "edges", "ragged"])
def test_morton_keys_bit_exact(dz, ctx, case):
    import torch
    L = 100.0
    if case == "uniform":
        ps = dzs_ics.uniform_random(5000, L, seed=1)
    elif case == "clustered":
        ps = dzs_ics.clustered_random(20001, L, seed=2, r_clump=0.3)
    elif case == "ragged":
        ps = dzs_ics.uniform_random(257, L, seed=3)
    else:
        v = np.array([0.0, np.nextafter(L, 0), 0.5 * L, np.nextafter(0.5 * L, 0), 1e-300, 25.0,
                      np.nextafter(25.0, 0), 12.5])
        g = np.stack(np.meshgrid(v, v, v, indexing="ij")).reshape(3, -1)
        ps = dzs_ics.uniform_random(g.shape[1], L, seed=4)
        ps.x, ps.y, ps.z = g[0].copy(), g[1].copy(), g[2].copy()
    _log(f"keys case={case} n={ps.n}")
    box, _ = _box(dz, L, ps.n, 32)
    st = dz.State.from_host(ps)
    keys = torch.zeros(ps.n, dtype=torch.int64, device="cuda")
    ctx.morton_keys(box, st, keys)
    torch.cuda.synchronize()
    got = keys.cpu().numpy().view(np.uint64)
    ref = oracle.morton_keys(ps.x, ps.y, ps.z, L)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("ties", [False, True])
def test_sort_state_is_stable_key_order(dz, ctx, ties):
    import torch
    L = 64.0
    ps = dzs_ics.clustered_random(30000, L, seed=5, r_clump=0.2)
    # duplicate some positions so equal keys occur
    rng = dzs_ics.rng(6)
    dup = rng.integers(0, ps.n, 500)
    ps.x[dup[1:]] = ps.x[dup[0]]
    ps.y[dup[1:]] = ps.y[dup[0]]
    ps.z[dup[1:]] = ps.z[dup[0]]
    ps.id = rng.permutation(ps.n).astype(np.uint32)
    _log(f"sort ties={ties} n={ps.n}")
    box, _ = _box(dz, L, ps.n, 32)
    st = dz.State.from_host(ps)
    perm = torch.zeros(ps.n, dtype=torch.int32, device="cuda")
    ctx.sort_state(box, st, ties_by_id=ties, perm=perm)
    torch.cuda.synchronize()
    out = st.to_host()
    p = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(p), np.arange(ps.n))
    keys = oracle.morton_keys(ps.x, ps.y, ps.z, L)
    if ties:
        ref = np.lexsort((ps.id, keys))
    else:
        ref = np.argsort(keys, kind="stable")
    assert np.array_equal(p, ref)
    for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
        assert np.array_equal(out[k], getattr(ps, k)[ref])


# ------------------------------------------------------------------------------- lightcone

def _lc_params(dz, fac, a0, a1, x_obs=(0.0, 0.0, 0.0)):
    sp = dz.step_factors(a0, a1, 0.3)
    lc = sp.lc
    # the selection scalars are shared inputs (oracle cosmology); the Chebyshev series used by
    # the crossing solve are the library's own
    lc.D = fac["D"]
    lc.chi2_0 = fac["chi2_0"]
    lc.chi2_1 = fac["chi2_1"]
    for d in range(3):
        lc.x_obs[d] = x_obs[d]
    return lc


@pytest.mark.parametrize("a0,a1,L", [(0.70, 0.74, 2000.0), (0.9247, 1.0, 600.0),
                                     (0.5, 0.52, 3000.0)])
def test_lightcone_emit_selection_bit_exact(dz, ctx, a0, a1, L):
    ps = dzs_ics.uniform_random(60000, L, seed=7, vel=1500.0)
    ps.id = dzs_ics.rng(8).permutation(ps.n).astype(np.uint32)
    fac = oracle.step_factors(a0, a1)
    lc = _lc_params(dz, fac, a0, a1)
    _log(f"lightcone a0={a0} a1={a1} L={L}")
    box, _ = _box(dz, L, ps.n, 40)
    st = dz.State.from_host(ps)
    ring = dz.LCRing(ps.n)
    ring.reset()
    ctx.lightcone_emit(box, st, lc, ring)
    rec = ring.records()
    mask, d0, _, _ = oracle.lightcone_select(ps.x, ps.y, ps.z, ps.px, ps.py, ps.pz, L,
                                             [0.0, 0.0, 0.0], fac["D"], fac["chi2_0"],
                                             fac["chi2_1"])
    assert rec["overflow"] == 0
    assert rec["count"] == int(mask.sum()) > 0
    assert np.array_equal(np.sort(rec["id"]), np.sort(ps.id[mask]))
    # crossing solve on a sample of records
    order = np.argsort(rec["id"])
    idx_by_id = {int(i): k for k, i in enumerate(ps.id)}
    for r in order[:: max(1, len(order) // 25)]:
        i = idx_by_id[int(rec["id"][r])]
        p = np.array([ps.px[i], ps.py[i], ps.pz[i]])
        ac = oracle.crossing_time(d0[:, i], p, a0, a1)
        assert abs(rec["a_cross"][r] - ac) <= 1e-12
        dref = d0[:, i] + p * oracle.drift_factor(a0, ac) if ac > a0 else d0[:, i]
        assert np.abs(rec["d"][r] - dref).max() <= 1e-9 * max(1.0, np.linalg.norm(dref))
        assert np.array_equal(rec["p"][r], p)
        assert rec["mult"][r] == ps.mult[i]


def test_lightcone_ring_overflow_flag(dz, ctx):
    L = 600.0
    ps = dzs_ics.uniform_random(20000, L, seed=9, vel=300.0)
    fac = oracle.step_factors(0.9247, 1.0)
    lc = _lc_params(dz, fac, 0.9247, 1.0)
    box, _ = _box(dz, L, ps.n, 27)
    st = dz.State.from_host(ps)
    ring = dz.LCRing(5)
    ring.reset()
    ctx.lightcone_emit(box, st, lc, ring)
    rec = ring.records()
    assert rec["overflow"] == 1 and rec["count"] > 5 and len(rec["id"]) == 5


# ----------------------------------------------------------------------------------- forces

def _force_case(kind, n, L, seed):
    if kind == "clustered":
        ps = dzs_ics.clustered_random(n, L, seed=seed, r_clump=L / 60)
    elif kind == "merged":
        ps = dzs_ics.merged_state(dzs_ics.clustered_random(n, L, seed=seed, r_clump=L / 40),
                                  seed=seed + 1, max_mult=64)
    else:
        ps = dzs_ics.zeldovich(round(n ** (1 / 3)), L, 0.02, seed=seed, spectrum="powerlaw")
    return ps


@pytest.mark.parametrize("kind,n", [("clustered", 20000), ("merged", 30001), ("zeldovich", 32768)])
def test_pm_force_matches_oracle(dz, ctx, kind, n):
    import torch
    L, ng = 100.0, 64
    r_s = 1.25 * L / ng
    ps = _force_case(kind, n, L, 11)
    _log(f"pm kind={kind} n={ps.n}")
    box, obox = _box(dz, L, ps.n, 32)
    st = dz.State.from_host(ps)
    ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP64, r_s, 0, 0))
    torch.cuda.synchronize()
    g = np.stack([st.gx[: ps.n].cpu().numpy(), st.gy[: ps.n].cpu().numpy(),
                  st.gz[: ps.n].cpu().numpy()])
    ref = oracle.pm_force(ps.x, ps.y, ps.z, ps.mult, obox, ng, r_s)
    err = _rms_rel(g, ref)
    _log(f"  pm rms rel err {err:.3e}")
    assert err <= 1e-8
    # deterministic: a second call gives the same bits
    ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP64, r_s, 0, 0))
    torch.cuda.synchronize()
    assert np.array_equal(st.gx[: ps.n].cpu().numpy(), g[0])


@pytest.mark.parametrize("kind,n,theta,tol,gsize", [("clustered", 20000, 0.0, 1e-10, 64),
                                                    ("merged", 30001, 0.0, 1e-10, 16),
                                                    ("zeldovich", 32768, 0.0, 1e-10, 8),
                                                    ("clustered", 20000, 0.0, 1e-10, 32),
                                                    ("clustered", 20000, 0.5, 5e-3, 16),
                                                    ("merged", 30001, 0.5, 5e-3, 64)])
def test_tree_force_matches_direct_sum(dz, ctx, kind, n, theta, tol, gsize):
    import torch
    L, ng = 100.0, 64
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    ps = _force_case(kind, n, L, 21)
    _log(f"tree kind={kind} n={ps.n} theta={theta} group={gsize}")
    box, obox = _box(dz, L, ps.n, 32)
    st = dz.State.from_host(ps)
    ctx.tree_force(box, st, dz.TreeParams(r_s, r_cut, theta, 8, gsize, dz.DZS_FP64, 0))
    torch.cuda.synchronize()
    g = np.stack([st.gx[: ps.n].cpu().numpy(), st.gy[: ps.n].cpu().numpy(),
                  st.gz[: ps.n].cpu().numpy()])
    ref = oracle.short_range(ps.x, ps.y, ps.z, ps.mult, obox, r_s, r_cut)
    err = _rms_rel(g, ref)
    _log(f"  tree rms rel err {err:.3e}")
    assert err <= tol
    ctx.tree_force(box, st, dz.TreeParams(r_s, r_cut, theta, 8, gsize, dz.DZS_FP64, 0))
    torch.cuda.synchronize()
    assert np.array_equal(st.gx[: ps.n].cpu().numpy(), g[0])


@pytest.mark.parametrize("kind,n,gsize", [("clustered", 20000, 16), ("merged", 30001, 64)])
def test_cell_start_walk_is_no_less_accurate_than_the_root_start(dz, ctx, kind, n, gsize):
    """The single-box walk starts at the level-K cells at least r_cut wide and always opens
    the nodes above them, some of which eq. 1 alone would accept as monopoles (a group box
    can sit up to r_cut + sqrt(3) l from a node's centre of mass).  The batched step walks
    from each box's root with eq. 1 at every level: at opening angle 0.5 both stay within the
    bar of the direct sum, and the cell start is the more accurate of the two."""
    import torch
    L, ng = 100.0, 64
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    ps = _force_case(kind, n, L, 27)
    _log(f"walk start kind={kind} n={ps.n} group={gsize}")
    box, obox = _box(dz, L, ps.n, 32)
    ref = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, obox, ng, r_s, r_cut)
    # cells: PM then the short range accumulated onto it
    st = dz.State.from_host(ps)
    ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP64, r_s, 0, 0))
    tp = dz.TreeParams(r_s, r_cut, 0.5, 8, gsize, dz.DZS_FP64, 0)
    tp.accumulate = 1
    ctx.tree_force(box, st, tp)
    torch.cuda.synchronize()
    g_cells = np.stack([st.gx[: ps.n].cpu().numpy(), st.gy[: ps.n].cpu().numpy(),
                        st.gz[: ps.n].cpu().numpy()])
    # root: a batch of this one box, with zero kick and drift factors
    st2 = dz.State.from_host(ps)
    sp = dz.step_factors(0.5, 0.51, 0.3)
    sp.K1 = sp.K2 = 0.0
    sp.lc.D = 0.0
    sp.do_lightcone, sp.do_coarsen = 0, 0
    sp.pm = dz.PMParams(0, dz.DZS_FP64, 0.0, 0, 0)
    sp.tree = dz.TreeParams(0.0, 0.0, 0.5, 8, gsize, dz.DZS_FP64, 0)
    ctx.kdk_step_batch([box], [0, ps.n], [ng], [r_s], [r_cut], st2, sp)
    torch.cuda.synchronize()
    ctx.check()
    h = st2.to_host()
    o = np.argsort(h["id"])
    assert np.array_equal(h["id"][o], np.sort(ps.id))
    r = np.argsort(ps.id)
    g_root = np.stack([h["gx"][o], h["gy"][o], h["gz"][o]])
    err_cells = _rms_rel(g_cells[:, r], ref[:, r])
    err_root = _rms_rel(g_root, ref[:, r])
    _log(f"  total force rms rel: cells {err_cells:.3e}, root {err_root:.3e}")
    # equal up to rounding when eq. 1 accepts no node above level K (the usual case)
    assert err_root <= 5e-3 and err_cells <= err_root * (1.0 + 1e-9)


@pytest.mark.parametrize("kind,n,gsize", [("clustered", 20000, 32), ("merged", 30001, 16)])
def test_tree_force_relative_opening(dz, ctx, kind, n, gsize):
    """Relative opening criterion (G M l^2 < alpha a_min d^4, a_min from the accelerations
    held on entry): alpha = 0 accepts no monopole and reproduces the opening-angle-0 walk bit
    for bit; a small alpha stays close to the oracle's direct sum, and the error and the
    interaction count move the right way with alpha.  The accelerations on entry are the
    oracle's PM + short-range force (the previous force of a run)."""
    import torch
    L, ng = 100.0, 64
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    ps = _force_case(kind, n, L, 23)
    _log(f"tree relative kind={kind} n={ps.n} group={gsize}")
    box, obox = _box(dz, L, ps.n, 32)
    ref = oracle.short_range(ps.x, ps.y, ps.z, ps.mult, obox, r_s, r_cut)
    g_old = ref + oracle.pm_force(ps.x, ps.y, ps.z, ps.mult, obox, ng, r_s)
    st = dz.State.from_host(ps)

    def run(alpha=None):
        for a, k in enumerate(("gx", "gy", "gz")):
            getattr(st, k)[: ps.n] = torch.from_numpy(np.ascontiguousarray(g_old[a]))
        tp = dz.TreeParams(r_s, r_cut, 0.0, 8, gsize, dz.DZS_FP64, 0)
        if alpha is not None:
            tp.opening, tp.alpha_open = dz.DZS_OPEN_RELATIVE, alpha
        ctx.pair_interactions(reset=True)
        ctx.tree_force(box, st, tp)
        torch.cuda.synchronize()
        g = np.stack([st.gx[: ps.n].cpu().numpy(), st.gy[: ps.n].cpu().numpy(),
                      st.gz[: ps.n].cpu().numpy()])
        return g, ctx.pair_interactions(reset=True)

    g_exact, p_exact = run()
    g0, p0 = run(0.0)
    assert np.array_equal(g0, g_exact) and p0 == p_exact
    scale = math.sqrt(np.mean(np.sum(g_old ** 2, axis=0)))
    errs, pairs = [], []
    for alpha in (0.05, 0.005, 0.0005):
        g, pr = run(alpha)
        e = math.sqrt(np.mean(np.sum((g - ref) ** 2, axis=0))) / scale
        _log(f"  alpha {alpha}: rms error / rms|g_old| {e:.3e}, interactions {pr} of {p_exact}")
        errs.append(e)
        pairs.append(pr)
    assert errs[0] <= 2e-2 and errs[2] <= 1e-3
    assert errs[0] >= errs[1] >= errs[2]
    assert pairs[0] <= pairs[1] <= pairs[2] <= p_exact and pairs[0] < p_exact


def test_tree_relative_opening_rejects(dz, ctx):
    import torch
    L = 100.0
    ps = dzs_ics.clustered_random(2000, L, seed=3)
    box, _ = _box(dz, L, ps.n, 12)
    st = dz.State.from_host(ps)
    for opening, alpha in ((2, 0.01), (dz.DZS_OPEN_RELATIVE, -1.0),
                           (dz.DZS_OPEN_RELATIVE, math.inf)):
        tp = dz.TreeParams(1.95, 8.8, 0.5, 8, 32, dz.DZS_FP64, 0)
        tp.opening, tp.alpha_open = opening, alpha
        with pytest.raises(dz.DZSError):
            ctx.tree_force(box, st, tp)
    torch.cuda.synchronize()


# Precision form: pair, mesh and FFT arithmetic in FP32 (unit roundoff 6e-8), positions and
# the accumulated force in FP64.  Bar: rms relative error <= 1e-5 against the FP64 oracle
# (the opening-angle-0 force bar; FP32 rounding of relative coordinates, ~1e-7 of r_cut,
# and of the FFT, ~log2(N_g^3) x 6e-8, stay well inside it).
@pytest.mark.parametrize("kind,n", [("clustered", 20000), ("merged", 30001), ("zeldovich", 32768)])
def test_pm_force_fp32_matches_oracle(dz, ctx, kind, n):
    import torch
    L, ng = 100.0, 64
    r_s = 1.25 * L / ng
    ps = _force_case(kind, n, L, 12)
    _log(f"pm fp32 kind={kind} n={ps.n}")
    box, obox = _box(dz, L, ps.n, 32)
    st = dz.State.from_host(ps)
    ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP32, r_s, 0, 0))
    torch.cuda.synchronize()
    g = np.stack([st.gx[: ps.n].cpu().numpy(), st.gy[: ps.n].cpu().numpy(),
                  st.gz[: ps.n].cpu().numpy()])
    ref = oracle.pm_force(ps.x, ps.y, ps.z, ps.mult, obox, ng, r_s)
    err = _rms_rel(g, ref)
    _log(f"  pm fp32 rms rel err {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("kind,n,theta,tol,gsize", [("clustered", 20000, 0.0, 1e-5, 64),
                                                    ("merged", 30001, 0.0, 1e-5, 16),
                                                    ("zeldovich", 32768, 0.0, 1e-5, 32),
                                                    ("zeldovich", 32768, 0.0, 1e-5, 64),
                                                    ("zeldovich", 32768, 0.0, 1e-5, 8),
                                                    ("clustered", 20000, 0.0, 1e-5, 4),
                                                    ("clustered", 20000, 0.5, 5e-3, 32),
                                                    ("clustered", 20000, 0.5, 5e-3, 64)])
def test_tree_force_fp32_matches_direct_sum(dz, ctx, kind, n, theta, tol, gsize):
    import torch
    L, ng = 100.0, 64
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    ps = _force_case(kind, n, L, 22)
    _log(f"tree fp32 kind={kind} n={ps.n} theta={theta} group={gsize}")
    box, obox = _box(dz, L, ps.n, 32)
    st = dz.State.from_host(ps)
    ctx.tree_force(box, st, dz.TreeParams(r_s, r_cut, theta, 8, gsize, dz.DZS_FP32, 0))
    torch.cuda.synchronize()
    g = np.stack([st.gx[: ps.n].cpu().numpy(), st.gy[: ps.n].cpu().numpy(),
                  st.gz[: ps.n].cpu().numpy()])
    ref = oracle.short_range(ps.x, ps.y, ps.z, ps.mult, obox, r_s, r_cut)
    err, n_flip, bounded = _fp32_force_error(g, ref, ps, obox, r_s, r_cut)
    _log(f"  tree fp32 rms rel err {err:.3e} (all targets {_rms_rel(g, ref):.3e}; "
         f"{n_flip} with a pair at r_cut)")
    assert err <= tol and (bounded or theta > 0)
    ctx.tree_force(box, st, dz.TreeParams(r_s, r_cut, theta, 8, gsize, dz.DZS_FP32, 0))
    torch.cuda.synchronize()
    assert np.array_equal(st.gx[: ps.n].cpu().numpy(), g[0])


@pytest.mark.parametrize("n", [0, 1, 2, 63, 65])
def test_force_tiny_inputs(dz, ctx, n):
    import torch
    L, ng = 50.0, 16
    r_s = 1.25 * L / ng
    ps = dzs_ics.uniform_random(max(n, 1), L, seed=30 + n)
    if n == 2:
        ps.x[1] = ps.x[0] + 1.0
        ps.y[1] = ps.y[0]
        ps.z[1] = ps.z[0]
    box, obox = _box(dz, L, max(n, 1), 4)
    st = dz.State.from_host(ps)
    st.n = n
    ctx.tree_force(box, st, dz.TreeParams(r_s, 4.5 * r_s, 0.0, 8, 64, dz.DZS_FP64, 0))
    ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP64, r_s, 1, 0))
    torch.cuda.synchronize()
    if n == 0:
        return
    g = np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(), st.gz[:n].cpu().numpy()])
    ref = oracle.short_range(ps.x[:n], ps.y[:n], ps.z[:n], ps.mult[:n], obox, r_s, 4.5 * r_s) + \
        oracle.pm_force(ps.x[:n], ps.y[:n], ps.z[:n], ps.mult[:n], obox, ng, r_s)
    lam = L / 4
    scale = obox.G * obox.m0 / lam ** 2      # natural force scale (the n = 1 force is ~0)
    assert np.abs(g - ref).max() <= 1e-8 * np.abs(ref).max() + 1e-10 * scale


# ------------------------------------------------------------------------------------- DZS

@pytest.mark.parametrize("case", range(5))
def test_coarsen_bit_exact(dz, ctx, case):
    import torch
    L = [100.0, 256.0, 1.0, 100.0, 50.0][case]
    n = [20000, 40000, 5000, 32768, 30000][case]
    if case == 3:
        ps = dzs_ics.zeldovich(32, L, 0.02, seed=20050528, spectrum="powerlaw")
        prm = dict(x_obs=[0.0, 0.0, 0.0], R_lc=20.0, b=5 * L / 32, theta=1.0, k_min=4)
    else:
        ps = dzs_ics.merged_state(dzs_ics.clustered_random(n, L, seed=40 + case, r_clump=L / 30,
                                                           vel=400.0), seed=case, max_mult=20)
        ps.id = dzs_ics.rng(50 + case).permutation(ps.n).astype(np.uint32)
        prm = dict(x_obs=[0.1 * L * case, 0.0, 0.3 * L], R_lc=0.15 * L, b=0.02 * L,
                   theta=[0.5, 1.0, 2.0, 0, 0.7][case], k_min=2 + case % 3)
    _log(f"coarsen case={case} n={ps.n}")
    res, group_of, nm = oracle.coarsen(ps, **prm)
    box, _ = _box(dz, L, ps.n, 32)
    st = dz.State.from_host(ps)
    cp = dz.CoarsenParams()
    for d in range(3):
        cp.x_obs[d] = prm["x_obs"][d]
    cp.R_lc, cp.b, cp.theta, cp.k_min = prm["R_lc"], prm["b"], prm["theta"], prm["k_min"]
    gof = torch.zeros(ps.n, dtype=torch.int32, device="cuda")
    rep = ctx.dzs_coarsen(box, st, cp, group_of=gof)
    torch.cuda.synchronize()
    out = st.to_host()
    assert nm > 0
    assert rep.n_groups == nm and rep.n_before == ps.n and rep.n_after == res["x"].shape[0]
    # the output is the (key, id) order on both sides: compare array for array, bit for bit
    for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
        assert np.array_equal(out[k], res[k]), k
    assert np.array_equal(gof.cpu().numpy().astype(np.int64), group_of)


@pytest.mark.parametrize("case", range(4))
def test_coarsen_dynamical_bit_exact(dz, ctx, case):
    """Dynamical criterion (eq. 2 with eq. 3): the same bit-exact bar as the geometric one,
    including the reduced a_min; case 3 puts nobody inside (a_min = +inf)."""
    import torch
    L = [100.0, 256.0, 1.0, 64.0][case]
    n = [20000, 40000, 7000, 12000][case]
    ps = dzs_ics.merged_state(dzs_ics.clustered_random(n, L, seed=70 + case, r_clump=L / 30,
                                                       vel=400.0), seed=case, max_mult=20)
    ps.id = dzs_ics.rng(80 + case).permutation(ps.n).astype(np.uint32)
    g = dzs_ics.rng(90 + case).standard_normal((3, ps.n)) * [1.0, 30.0, 1e-3, 5.0][case]
    box, obox = _box(dz, L, ps.n, 32)
    R = 0.0 if case == 3 else 0.15 * L
    b = 1e-9 * L if case == 3 else 0.02 * L
    prm = dict(x_obs=[0.1 * L * case, 0.0, 0.3 * L], R_lc=R, b=b, theta=None, k_min=2 + case % 3,
               alpha_dyn=[3e-2, 1e-3, 1.0, 1e-6][case])
    _log(f"coarsen dynamical case={case} n={ps.n}")
    res, group_of, nm = oracle.coarsen(ps, **prm, g=g, Gm0=obox.G * obox.m0)
    st = dz.State.from_host(ps, g=g)
    cp = dz.CoarsenParams()
    for d in range(3):
        cp.x_obs[d] = prm["x_obs"][d]
    cp.R_lc, cp.b, cp.k_min = prm["R_lc"], prm["b"], prm["k_min"]
    cp.criterion, cp.alpha_dyn = dz.DZS_CRIT_DYNAMICAL, prm["alpha_dyn"]
    gof = torch.zeros(ps.n, dtype=torch.int32, device="cuda")
    rep = ctx.dzs_coarsen(box, st, cp, group_of=gof)
    torch.cuda.synchronize()
    out = st.to_host()
    assert nm > 0 and 0 < res["x"].shape[0] < ps.n
    assert rep.a_min == res["a_min"]
    if case == 3:
        assert rep.a_min == math.inf
    assert rep.n_groups == nm and rep.n_after == res["x"].shape[0]
    for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
        assert np.array_equal(out[k], res[k]), k
    assert np.array_equal(gof.cpu().numpy().astype(np.int64), group_of)


def test_coarsen_dynamical_zero_alpha_and_rejects(dz, ctx):
    import torch
    L = 100.0
    ps = dzs_ics.clustered_random(8000, L, seed=61)
    g = dzs_ics.rng(62).standard_normal((3, ps.n))
    box, _ = _box(dz, L, ps.n, 20)
    st = dz.State.from_host(ps, g=g)
    cp = dz.CoarsenParams()
    cp.R_lc, cp.b, cp.k_min = 10.0, 1.0, 2
    cp.criterion, cp.alpha_dyn = dz.DZS_CRIT_DYNAMICAL, 0.0
    rep = ctx.dzs_coarsen(box, st, cp)
    torch.cuda.synchronize()
    assert rep.n_groups == 0 and st.n == ps.n and rep.a_min > 0
    for bad in (dict(criterion=2), dict(alpha_dyn=-1.0), dict(alpha_dyn=math.inf)):
        cp2 = dz.CoarsenParams()
        cp2.R_lc, cp2.b, cp2.k_min = 10.0, 1.0, 2
        cp2.criterion, cp2.alpha_dyn = dz.DZS_CRIT_DYNAMICAL, 1.0
        for k, v in bad.items():
            setattr(cp2, k, v)
        with pytest.raises(dz.DZSError):
            ctx.dzs_coarsen(box, st, cp2)
    # the geometric criterion still needs theta > 0
    cp3 = dz.CoarsenParams()
    cp3.R_lc, cp3.b, cp3.k_min, cp3.theta = 10.0, 1.0, 2, 0.0
    with pytest.raises(dz.DZSError):
        ctx.dzs_coarsen(box, st, cp3)


def test_coarsen_no_merge_region_is_identity(dz, ctx):
    import torch
    L = 100.0
    ps = dzs_ics.clustered_random(10000, L, seed=60)
    box, _ = _box(dz, L, ps.n, 22)
    st = dz.State.from_host(ps)
    cp = dz.CoarsenParams()
    cp.R_lc, cp.b, cp.theta, cp.k_min = math.sqrt(3) / 2 * L, 0.0, 10.0, 1
    rep = ctx.dzs_coarsen(box, st, cp)
    torch.cuda.synchronize()
    out = st.to_host()
    assert rep.n_groups == 0 and st.n == ps.n
    o = np.argsort(out["id"])
    assert np.array_equal(out["x"][o], ps.x[np.argsort(ps.id)])


# -------------------------------------------------------------------------------- KDK step

@pytest.mark.parametrize("coarsen,fp32", [(False, False), (True, False), (True, True),
                                           ("dyn", False), ("relative-opening", False)])
def test_kdk_step_matches_oracle(dz, ctx, coarsen, fp32):
    """One step of the 32^3 box: Zel'dovich at z = 49, L = 100, mesh 64.  In the precision form
    the drift, the coarsening and the lightcone test stay FP64 (bit-exact); the force and the
    momenta carry the FP32 force bar, 1e-5."""
    import torch
    L, ng, n_side = 100.0, 64, 32
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    ps = dzs_ics.zeldovich(n_side, L, 0.02, seed=20050528, spectrum="powerlaw")
    box, obox = _box(dz, L, ps.n, n_side)
    g0 = oracle.total_force(ps.x, ps.y, ps.z, ps.mult, obox, ng, r_s, r_cut)
    a0, a1 = 0.02, 0.02 * math.exp(0.07824)
    fac = oracle.step_factors(a0, a1)
    fac.update(a0=a0, a1=a1)
    rel_open = coarsen == "relative-opening"
    if rel_open:
        coarsen = False
    cparams = dict(R_lc=20.0, b=5 * L / n_side, theta=1.0, k_min=4) if coarsen else None
    if coarsen == "dyn":
        # dynamical criterion on the previous (initial) force; alpha = 0.3 merges ~1000 nodes
        cparams.update(theta=None, alpha_dyn=0.3)
    _log(f"kdk coarsen={coarsen} fp32={fp32}")
    prec = dz.DZS_FP32 if fp32 else dz.DZS_FP64
    tol = 1e-5 if fp32 else 1e-9
    ref_state, ref_g, _, cres = oracle.kdk_step(ps, g0, obox, fac, ng, r_s, r_cut,
                                                [0.0, 0.0, 0.0], coarsen_params=cparams,
                                                solve=False)
    sp = dz.step_factors(a0, a1, 0.3)
    sp.K1, sp.K2 = fac["K1"], fac["K2"]
    sp.lc.D, sp.lc.chi2_0, sp.lc.chi2_1 = fac["D"], fac["chi2_0"], fac["chi2_1"]
    sp.do_lightcone = 1
    sp.do_coarsen = 1 if coarsen else 0
    if coarsen:
        sp.coarsen.R_lc, sp.coarsen.b = cparams["R_lc"], cparams["b"]
        sp.coarsen.k_min = cparams["k_min"]
        if coarsen == "dyn":
            sp.coarsen.criterion = dz.DZS_CRIT_DYNAMICAL
            sp.coarsen.alpha_dyn = cparams["alpha_dyn"]
        else:
            sp.coarsen.theta = cparams["theta"]
    sp.pm = dz.PMParams(ng, prec, r_s, 0, 0)
    sp.tree = dz.TreeParams(r_s, r_cut, 0.0, 8, 64, prec, 0)
    if rel_open:
        # monopoles accepted by G M l^2 < alpha |g_0|_min d^4 on the entry force g0
        sp.tree.opening, sp.tree.alpha_open = dz.DZS_OPEN_RELATIVE, 1e-3
        tol = 2e-3
    st = dz.State.from_host(ps, g=g0)
    ring = dz.LCRing(1000)
    ring.reset()
    rep = ctx.kdk_step(box, st, sp, ring)
    torch.cuda.synchronize()
    out = st.to_host()
    assert st.n == ref_state.n
    if coarsen:
        assert rep.n_groups == cres[2] > 0
    if coarsen == "dyn":
        assert rep.a_min == cres[0]["a_min"]
    o = np.argsort(out["id"])
    r = np.argsort(ref_state.id)
    # positions after the drift (and the coarsening) are bit-exact
    for k in ("x", "y", "z", "mult", "id", "type"):
        assert np.array_equal(out[k][o], getattr(ref_state, k)[r]), k
    gg = np.stack([out["gx"][o], out["gy"][o], out["gz"][o]])
    err = _rms_rel(gg, ref_g[:, r])
    _log(f"  kdk g rms rel err {err:.3e}")
    if fp32:
        # FP32 rounding is relative to the parts summed, not to their near-cancelling total
        # (a z = 49 lattice): normalise by the rms of |g_PM| + |g_short|
        g_pm = oracle.pm_force(ref_state.x, ref_state.y, ref_state.z, ref_state.mult, obox, ng,
                               r_s)
        g_sr = oracle.short_range(ref_state.x, ref_state.y, ref_state.z, ref_state.mult, obox,
                                  r_s, r_cut)
        parts = np.sqrt((g_pm ** 2).sum(0)) + np.sqrt((g_sr ** 2).sum(0))
        err, n_flip, bounded = _fp32_force_error(gg, ref_g[:, r], ref_state.take(r), obox, r_s,
                                                 r_cut, norm=parts)
        _log(f"  kdk g rms err / rms(|g_PM| + |g_short|) {err:.3e}, {n_flip} targets with a "
             f"pair at r_cut")
        assert bounded
    assert err <= tol
    for a, k in enumerate(("px", "py", "pz")):
        scale = np.abs(getattr(ref_state, k)).max()
        dp = out[k][o] - getattr(ref_state, k)[r]
        if fp32 or rel_open:
            # the closing kick is FP64: the momentum differs by exactly K2 times the force
            # difference checked above (which may hold a cutoff flip or monopoles)
            dp = dp - fac["K2"] * (gg[a] - ref_g[a, r])
        assert np.abs(dp).max() <= 1e-9 * scale
    assert ring.records()["count"] == 0   # chi(z=49) >> L: no particle on the lightcone


@pytest.mark.parametrize("coarsen", [False, True])
def test_lightcone_emits_every_particle_once_over_a_run(dz, ctx, coarsen):
    """A 32^3 box (L = 1000, observer at the corner) run through 50 log steps to z = 0: the
    shrinking sphere passes every particle once, so every id is emitted exactly once with its
    own multiplicity 1; with DZS the merged particles lie outside the sphere when they form
    and never cross again."""
    import torch
    n_side, L, ng = 32, 1000.0, 64
    ps = dzs_ics.zeldovich(n_side, L, 0.02, seed=20050533, spectrum="bbks")
    lam = L / n_side
    box, _ = _box(dz, L, ps.n, n_side)
    r_s = 1.25 * L / ng
    a = np.exp(np.linspace(math.log(0.02), 0.0, 51))
    st = dz.State.from_host(ps)
    ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP64, r_s, 0, 0))
    ctx.tree_force(box, st, dz.TreeParams(r_s, 4.5 * r_s, 0.5, 8, 32, dz.DZS_FP64, 1))
    ring = dz.LCRing(2 * ps.n)
    ring.reset()
    merged = 0
    for s in range(50):
        sp = dz.step_factors(float(a[s]), float(a[s + 1]), 0.3)
        sp.do_lightcone = 1
        sp.do_coarsen = 1 if (coarsen and s < 49) else 0
        sp.coarsen.R_lc = math.sqrt(sp.lc.chi2_1)
        sp.coarsen.b, sp.coarsen.theta, sp.coarsen.k_min = 5 * lam, 1.0, 4
        sp.pm = dz.PMParams(ng, dz.DZS_FP64, r_s, 0, 0)
        sp.tree = dz.TreeParams(r_s, 4.5 * r_s, 0.5, 8, 32, dz.DZS_FP64, 0)
        merged += int(ctx.kdk_step(box, st, sp, ring).n_groups)
    torch.cuda.synchronize()
    rec = ring.records()
    _log(f"lightcone run coarsen={coarsen}: {rec['count']} records, merged nodes {merged}, "
         f"final n {st.n}")
    assert rec["overflow"] == 0
    if coarsen:
        assert merged > 0 and st.n < ps.n
    ids = np.sort(rec["id"])
    assert np.array_equal(ids, np.sort(ps.id))
    assert np.all(rec["mult"] == 1)
    assert np.all((rec["a_cross"] >= 0.02) & (rec["a_cross"] <= 1.0))


def test_fp32_mesh_context_matches_and_rejects_plain_pm(dz):
    """A context whose meshes are sized for the precision form only (the deposit shares the
    complex mesh) gives the same FP32 PM force bit for bit, and refuses the plain form."""
    import torch
    L, ng = 100.0, 64
    r_s = 1.25 * L / ng
    ps = _force_case("clustered", 20000, L, 13)
    box, _ = _box(dz, L, ps.n, 32)
    out = []
    for flag in (False, True):
        c = dz.Context(max_particles=ps.n, max_mesh_side=ng, fp32_meshes=flag)
        st = dz.State.from_host(ps)
        c.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP32, r_s, 0, 0))
        torch.cuda.synchronize()
        out.append(np.stack([st.gx[: ps.n].cpu().numpy(), st.gy[: ps.n].cpu().numpy()]))
        if flag:
            with pytest.raises(dz.DZSError):
                c.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP64, r_s, 0, 0))
        c.close()
    assert np.array_equal(out[0], out[1])

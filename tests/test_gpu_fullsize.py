"""Parity at the full sizes of the benchmark workloads, in the launch configuration bench.py
times (tree opening angle 0.5, 32 targets per group, leaves of 16 at 128^3 and 8 at 512^3
and 1024^3, the default PM tiles), on sampled outputs.

The GPU computes the force of every particle (at 1024^3: of the sampled targets, through
tree_force's target subset); the oracle computes it for a seeded sample of targets: the PM
part on the full mesh (deposit of every particle, Poisson solve, 4-point gradient)
interpolated at the sampled targets, and the short-range part as the direct sum over every
source within r_cut of each sampled target (sources found by binning the box in cells at
least r_cut wide, or at 1024^3 by lattice index, so the sum is complete).

  128^3, L = 256, mesh 256^3, FP64 plain form, at z = 49 and on a clustered late state
  512^3, L = 1000, mesh 512^3, FP32 precision form, at z = 49 and on a clustered late state
  1024^3, L = 2000, mesh 1024^3, FP32 precision form at z = 49 (the headline's start): the
      short range against the oracle; the PM against the GPU's FP64 plain-form PM (a 1024^3
      FP64 mesh solve does not fit the oracle's test budget), which the 128^3 and 512^3 cases
      hold to the oracle's PM

The clustered late states are the seeded Zel'dovich approximation evaluated at a = 1 (the
input generator's, shared by both sides): shell-crossed sheets and filaments that give the
tree its depth, wide groups and dense leaves.
"""
import math
import sys

import numpy as np
import pytest

import dzs_ics
import oracle

pytestmark = pytest.mark.gpu

CASES = {
    "128cube_fp64": dict(n_side=128, L=256.0, ng=256, seed=20050529, fp32=False, n_t=1500,
                         leaf=16, a=0.02),
    "128cube_fp64_late": dict(n_side=128, L=256.0, ng=256, seed=20050529, fp32=False,
                              n_t=1500, leaf=16, a=1.0),
    "512cube_fp32": dict(n_side=512, L=1000.0, ng=512, seed=20050530, fp32=True, n_t=600,
                         leaf=8, a=0.02),
    "512cube_fp32_late": dict(n_side=512, L=1000.0, ng=512, seed=20050530, fp32=True, n_t=600,
                              leaf=8, a=1.0),
}


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _neighbour_sources(ps, targets, r_cut):
    """Indices of every particle within r_cut (minimum image) of any sampled target, and the
    per-target flag of a source within 1e-5 r_cut of the cutoff (FP32 may keep or drop it)."""
    L = ps.L
    nc = max(3, int(L // r_cut))
    cs = L / nc
    ix = np.minimum((ps.x / cs).astype(np.int64), nc - 1)
    iy = np.minimum((ps.y / cs).astype(np.int64), nc - 1)
    iz = np.minimum((ps.z / cs).astype(np.int64), nc - 1)
    cell = (ix * nc + iy) * nc + iz
    order = np.argsort(cell, kind="stable")
    starts = np.searchsorted(cell[order], np.arange(nc ** 3 + 1))
    cand, near_cut = [], np.zeros(targets.size, bool)
    for t_i, t in enumerate(targets):
        cx, cy, cz = ix[t], iy[t], iz[t]
        ids = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz_ in (-1, 0, 1):
                    c = ((((cx + dx) % nc) * nc + (cy + dy) % nc) * nc + (cz + dz_) % nc)
                    ids.append(order[starts[c]:starts[c + 1]])
        ids = np.unique(np.concatenate(ids))
        d = [getattr(ps, k)[ids] - getattr(ps, k)[t] for k in ("x", "y", "z")]
        d = [v - L * np.round(v / L) for v in d]
        r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        near_cut[t_i] = bool(np.any(np.abs(r - r_cut) < 1e-5 * r_cut))
        cand.append(ids[r < r_cut * (1 + 1e-9)])
    return np.unique(np.concatenate(cand + [targets])), near_cut


@pytest.mark.timeout(400)
@pytest.mark.parametrize("name", list(CASES))
def test_full_size_force_on_sampled_targets(name):
    import torch

    import paper_2005_05328_amd as dz
    c = CASES[name]
    L, ng, n_side = c["L"], c["ng"], c["n_side"]
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    lam = L / n_side
    _log(f"full size {name}: {n_side}^3, L={L}, mesh {ng}")
    ps = dzs_ics.zeldovich(n_side, L, c["a"], seed=c["seed"], spectrum="bbks")
    n = ps.n
    m0 = dzs_ics.particle_mass(L, n)
    box = dz.make_box(L, m0, lam / 40)
    obox = oracle.Box(L=L, m0=m0, eps0=lam / 40)
    prec = dz.DZS_FP32 if c["fp32"] else dz.DZS_FP64
    ctx = dz.Context(n, ng)
    st = dz.State.from_host(ps)
    # PM alone, then PM + the tree as the benchmark's step computes them
    if c["fp32"]:
        # the plain-form PM, the reference of the 1024^3 case, against the oracle here too
        ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP64, r_s, 0, 0))
        torch.cuda.synchronize()
        g_pm64 = np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(),
                           st.gz[:n].cpu().numpy()])
    ctx.pm_force(box, st, dz.PMParams(ng, prec, r_s, 0, 0))
    torch.cuda.synchronize()
    g_pm = np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(), st.gz[:n].cpu().numpy()])
    ctx.tree_force(box, st, dz.TreeParams(r_s, r_cut, 0.5, c["leaf"], 32, prec, 1))
    torch.cuda.synchronize()
    g_all = np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(), st.gz[:n].cpu().numpy()])
    ctx.tree_force(box, st, dz.TreeParams(r_s, r_cut, 0.0, c["leaf"], 32, prec, 0))
    torch.cuda.synchronize()
    g_sr0 = np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(), st.gz[:n].cpu().numpy()])
    ctx.close()
    del st
    _log("  GPU forces done")

    t = np.sort(dzs_ics.rng(c["seed"] + 7).choice(n, c["n_t"], replace=False))
    # oracle PM at the targets
    rho = oracle.cic_deposit(ps.x, ps.y, ps.z, ps.mult, L, ng, m0)
    psi = oracle.pm_potential(rho, L, r_s, obox.G)
    del rho
    ref_pm = np.stack([oracle.cic_interp(ps.x[t], ps.y[t], ps.z[t], L, gm)
                       for gm in oracle.fd4_gradient(psi, L)])
    del psi
    # oracle short range at the targets from every source within r_cut
    src, near_cut = _neighbour_sources(ps, t, r_cut)
    pos = np.searchsorted(src, t)
    ref_sr = oracle.short_range(ps.x[src], ps.y[src], ps.z[src], ps.mult[src], obox, r_s, r_cut,
                                targets=pos)
    _log(f"  oracle done: {t.size} targets, {src.size} sources, {int(near_cut.sum())} targets "
         f"with a source within 1e-5 r_cut of the cutoff")

    # FP32 rounding is relative to the parts summed, not to their near-cancelling total (a
    # z = 49 lattice): the precision form is scaled by |g_PM| + |g_short| per target
    parts = np.sqrt((ref_pm ** 2).sum(0)) + np.sqrt((ref_sr ** 2).sum(0))

    def rms_rel(g, ref, keep=None, by_parts=c["fp32"]):
        keep = np.ones(ref.shape[1], bool) if keep is None else keep
        num = np.mean(np.sum((g[:, keep] - ref[:, keep]) ** 2, axis=0))
        scale2 = parts[keep] ** 2 if by_parts else np.sum(ref[:, keep] ** 2, axis=0)
        return math.sqrt(num / np.mean(scale2))

    e_pm = rms_rel(g_pm[:, t], ref_pm)
    if c["fp32"]:
        e_pm64 = rms_rel(g_pm64[:, t], ref_pm, by_parts=False)
        _log(f"  plain-form PM rms rel {e_pm64:.3e}")
        assert e_pm64 <= 1e-8
    e_sr0 = rms_rel(g_sr0[:, t], ref_sr, ~near_cut if c["fp32"] else None)
    # the opening-angle error, like rounding, is relative to the parts summed
    e_all = rms_rel(g_all[:, t], ref_pm + ref_sr, by_parts=True)
    _log(f"  PM rms rel {e_pm:.3e}; short range (theta 0) {e_sr0:.3e}; "
         f"total at theta 0.5 {e_all:.3e}")
    # the plain form's bars of the small-size tests: PM 1e-8 (32.32 fixed-point deposit),
    # exact short range 1e-9; the precision form's 1e-5
    assert e_pm <= (1e-5 if c["fp32"] else 1e-8)
    assert e_sr0 <= (1e-5 if c["fp32"] else 1e-9)
    # the targets set aside must stay a small part of the sample (clustered states hold more
    # pairs near the cutoff: 31 of 600 at 512^3)
    assert near_cut.sum() <= 0.1 * t.size
    assert e_all <= 5e-3


def _lattice_sources(n_side, targets, r_cut, lam):
    """Indices of every lattice particle whose lattice site is within r_cut + 2 lambda of a
    target's site (per axis, periodic): a superset of the sources within r_cut while every
    displacement is below half a lattice cell."""
    pad = int(math.ceil(r_cut / lam)) + 2
    off = np.arange(-pad, pad + 1)
    i, j, k = np.unravel_index(targets, (n_side,) * 3)
    out = []
    for t in range(targets.size):
        ax = [(v + off) % n_side for v in (i[t], j[t], k[t])]
        out.append(((ax[0][:, None, None] * n_side + ax[1][None, :, None]) * n_side
                    + ax[2][None, None, :]).ravel())
    return np.unique(np.concatenate(out))


@pytest.mark.timeout(900)
def test_full_size_1024cube_on_sampled_targets():
    """The headline configuration: 1024^3 particles, L = 2000, mesh 1024^3, FP32 precision
    form, opening angle 0.5, groups of 64, leaves of 8, on the z = 49 initial state, in a
    context of the headline's memory plan but with plain-form-capable meshes.  The state is
    sorted once; the short range of 600 sampled targets (tree_force's target subset on the
    presorted state) against the oracle's direct sum, and the PM against the GPU's FP64 PM."""
    import torch

    import paper_2005_05328_amd as dz
    n_side, L, ng, seed = 1024, 2000.0, 1024, 20050532
    r_s = 1.25 * L / ng
    r_cut = 4.5 * r_s
    lam = L / n_side
    _log(f"full size 1024^3: L={L}, mesh {ng}")
    ps = dzs_ics.zeldovich(n_side, L, 1.0 / 50.0, seed=seed, spectrum="bbks")
    assert ps.max_disp < 0.5 * lam
    n = ps.n
    m0 = dzs_ics.particle_mass(L, n)
    box = dz.make_box(L, m0, lam / 40)
    obox = oracle.Box(L=L, m0=m0, eps0=lam / 40)
    sample = np.sort(dzs_ics.rng(seed + 7).choice(n, 600, replace=False)).astype(np.int64)
    ctx = dz.Context(n, ng, no_copies=True)
    st = dz.State.from_host(ps)
    _log("  state resident")
    ctx.sort_state(box, st)
    # slots of the sampled ids in the sorted state (ids are lattice indices)
    flag = torch.zeros(n, dtype=torch.bool, device="cuda")
    flag[torch.from_numpy(sample).cuda()] = True
    slots = torch.nonzero(flag.index_select(0, st.id[:n])).flatten().to(torch.int32)
    del flag
    t_ids = st.id[slots.to(torch.int64)].cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(t_ids), sample)

    def at_targets():
        torch.cuda.synchronize()
        sl = slots.to(torch.int64)
        return np.stack([st.gx[sl].cpu().numpy(), st.gy[sl].cpu().numpy(),
                         st.gz[sl].cpu().numpy()])

    ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP64, r_s, 0, 0))
    g_pm64 = at_targets()
    ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP32, r_s, 0, 0))
    g_pm = at_targets()
    tp = dz.TreeParams(r_s, r_cut, 0.0, 8, 64, dz.DZS_FP32, 0)
    tp.presorted = 1
    ctx.tree_force(box, st, tp, targets=slots)
    ctx.check()
    g_sr0 = at_targets()
    ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP32, r_s, 0, 0))
    tp = dz.TreeParams(r_s, r_cut, 0.5, 8, 64, dz.DZS_FP32, 1)
    tp.presorted = 1
    ctx.tree_force(box, st, tp, targets=slots)
    ctx.check()
    g_all = at_targets()
    ctx.close()
    del st
    _log("  GPU forces done")
    src = _lattice_sources(n_side, t_ids, r_cut, lam)
    tpos = np.searchsorted(src, t_ids)
    ref_sr = oracle.short_range(ps.x[src], ps.y[src], ps.z[src], ps.mult[src], obox, r_s, r_cut,
                                targets=tpos)
    # pairs within FP32 rounding of r_cut may be kept or dropped: flag their targets
    near_cut = np.zeros(t_ids.size, bool)
    for q, i in enumerate(t_ids):
        d = [getattr(ps, k)[src] - getattr(ps, k)[i] for k in ("x", "y", "z")]
        d = [v - L * np.round(v / L) for v in d]
        r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        near_cut[q] = bool(np.any(np.abs(r - r_cut) < 1e-5 * r_cut))
    _log(f"  oracle done: {src.size} sources, {int(near_cut.sum())} targets near the cutoff")
    parts = np.sqrt((g_pm64 ** 2).sum(0)) + np.sqrt((ref_sr ** 2).sum(0))

    def rms(g, ref, keep=None):
        keep = np.ones(ref.shape[1], bool) if keep is None else keep
        num = np.mean(np.sum((g[:, keep] - ref[:, keep]) ** 2, axis=0))
        return math.sqrt(num / np.mean(parts[keep] ** 2))

    e_pm = rms(g_pm, g_pm64)
    e_sr0 = rms(g_sr0, ref_sr, ~near_cut)
    e_all = rms(g_all, g_pm64 + ref_sr)
    _log(f"  PM FP32 vs FP64 {e_pm:.3e}; short range (theta 0) {e_sr0:.3e}; total at theta "
         f"0.5 {e_all:.3e}")
    assert e_pm <= 1e-5 and e_sr0 <= 1e-5
    assert near_cut.sum() <= 0.1 * t_ids.size
    assert e_all <= 5e-3

#!/usr/bin/env python3
"""Benchmark of the MI355X DZS gravity step.

Default workload (the 128^3 configuration, `--workload c2`): 128^3 particles, periodic box
L = 256 Mpc/h, PM mesh 256^3, split scale r_s = 1.25 mesh cells, cutoff 4.5 r_s, Zel'dovich start
at z = 49 from a seeded Gaussian random field with a LCDM-shaped (BBKS, Omega_m = 0.3,
sigma_8 = 0.8) spectrum, observer at the box corner, 50 log-spaced KDK steps to z = 0, all in
the FP64 plain form.  Each step is one kdk_step call: kick, drift + lightcone crossing output,
DZS coarsening (2x2x2, theta = 0.1, b = 5 lambda, l_max = 2 lambda; the host check skips the
merge kernels at boundaries where no node can qualify), Morton sort, tree build, PM force,
tree force (opening angle 0.5), kick.

value = particle force updates per second = N * K / wall time of the K timed steps (inputs
resident in HBM; the timed region is bracketed by torch.cuda.synchronize()).  A twin run
follows: the full-resolution run (no DZS) for the DZS/full-resolution wall-time ratio and the
lightcone comparison, or (`--workload c3`) the FP64 plain form against the timed precision
form, with force errors at the initial and final states.

Other workloads: c3 = 512^3, L = 1000, mesh 512^3, precision form vs plain form (l_max =
4 lambda); c5s = 256^3, L = 2000, mesh 256^3, 100 steps, precision form, DZS vs full
resolution (the DZS geometry of the 1024^3 configuration at lower resolution); c5 = 1024^3,
L = 2000, mesh 1024^3, 100 steps (use --steps to bound it).

Prints ONE JSON line.  `--gpus N` with N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "particle force updates/sec on 1 GPU; DZS vs full-res wall time at equal accuracy"
UNIT = "particle force updates/s"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
FLOP_PER_INTERACTION = 24

ROOT = os.path.dirname(os.path.abspath(__file__))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# workload presets: particles per side, box, mesh, seed, steps, l_max / lambda, form, twin
PRESETS = {
    "c2": dict(n_side=128, L=256.0, ng=256, seed=20050529, n_steps=50, lmax_over_lambda=2,
               precision="fp64", twin="dzs"),
    # leaves of 8 for the large clustered runs (the 512^3 run's walk: 310 ms per launch
    # against 330 with leaves of 16); 16 at 128^3
    "c3": dict(n_side=512, L=1000.0, ng=512, seed=20050530, n_steps=50, lmax_over_lambda=4,
               precision="fp32", twin="precision", leaf=8),
    "c5s": dict(n_side=256, L=2000.0, ng=256, seed=20050532, n_steps=100, lmax_over_lambda=4,
                precision="fp32", twin="dzs", leaf=8),
    "c5": dict(n_side=1024, L=2000.0, ng=1024, seed=20050532, n_steps=100, lmax_over_lambda=4,
               precision="fp32", twin="dzs", leaf=8),
    # the 64-box ensemble: run by run_ensemble(), not by the single-box path
    "c4": dict(n_side=0, L=0.0, ng=0, seed=20051000, n_steps=10, lmax_over_lambda=0,
               precision="fp32", twin=None),
}


def ensemble_boxes():
    """The 64-box ensemble: box i has side 128 + 256 (i mod 8) / 7 Mpc/h, 32^3, 48^3, 64^3 or
    96^3 particles (i // 16), a mesh of twice the particles per side, seed 20051000 + i, and is
    coarsened once at DZS level 1 + (i mod 3) (l_max = 2^level lambda)."""
    out = []
    for i in range(64):
        n_side = [32, 48, 64, 96][i // 16]
        L = 128.0 + 256.0 * (i % 8) / 7.0
        out.append(dict(i=i, n_side=n_side, L=L, ng=2 * n_side, seed=20051000 + i,
                        level=1 + i % 3))
    return out


def run_ensemble(args, dz, torch, dzs_ics):
    """Config 4: 64 independent boxes (Zel'dovich at z = 9), each coarsened once outside a
    prescribed lightcone radius R_lc = L/4 (theta 1, b = 0, l_max = 2^level lambda), then
    advanced together by kdk_step_batch in the precision form; the same steps run box by box
    with kdk_step for the launch-overhead comparison.  A short autotuning pass picks the
    walk's group and leaf sizes first."""
    K = max(1, min(args.steps or 10, 10))
    prec = dz.DZS_FP64 if args.precision == "fp64" else dz.DZS_FP32
    a = np.exp(np.linspace(math.log(0.1), math.log(0.1) + 0.05 * 10, 11))
    specs = ensemble_boxes()
    big = max(sp_["n_side"] for sp_ in specs) ** 3
    cctx = dz.Context(big, 2 * max(sp_["n_side"] for sp_ in specs))
    parts, boxes, first, ngs, rss, rcs = [], [], [0], [], [], []
    id_base = 0
    log("ensemble: initial conditions and per-box coarsening")
    for b in specs:
        ps = dzs_ics.zeldovich(b["n_side"], b["L"], 0.1, seed=b["seed"], spectrum="bbks")
        lam = b["L"] / b["n_side"]
        m0 = dzs_ics.particle_mass(b["L"], ps.n)
        box = dz.make_box(b["L"], m0, lam / 40)
        st = dz.State.from_host(ps)
        cp = dz.CoarsenParams()
        cp.R_lc, cp.b, cp.theta = 0.25 * b["L"], 0.0, 1.0
        cp.k_min = k_min_for(b["n_side"], 2 ** b["level"])
        cctx.dzs_coarsen(box, st, cp)
        torch.cuda.synchronize()
        h = st.to_host()
        h["id"] = h["id"] + np.uint32(id_base)
        id_base += b["n_side"] ** 3
        parts.append(h)
        boxes.append(box)
        first.append(first[-1] + h["x"].shape[0])
        ngs.append(b["ng"])
        rss.append(1.25 * b["L"] / b["ng"])
        rcs.append(4.5 * 1.25 * b["L"] / b["ng"])
    cctx.close()
    N = first[-1]
    log(f"ensemble: {N} particles in 64 boxes after coarsening "
        f"({sum(sp_['n_side'] ** 3 for sp_ in specs)} before)")

    class _P:
        pass
    allp = _P()
    for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
        setattr(allp, k, np.concatenate([h[k] for h in parts]))
    cells = sum(g ** 3 for g in ngs)
    side = 8
    while side ** 3 < cells or not _smooth(side):
        side += 1
    ctx = dz.Context(N + 64, side)
    st0 = dz.State.from_host(allp, capacity=N + 64)
    st = dz.State(N + 64)
    ring = dz.LCRing(1024)

    def params(s_, group, leaf, chunk=0):
        sp_ = dz.step_factors(float(a[s_]), float(a[s_ + 1]), 0.3)
        sp_.do_lightcone, sp_.do_coarsen = 1, 0
        sp_.pm = dz.PMParams(0, prec, 0.0, 0, chunk)
        sp_.tree = dz.TreeParams(0.0, 0.0, 0.5, leaf, group, prec, 0)
        return sp_

    def batch_run(steps, group, leaf, chunk=0):
        copy_state(st, st0)
        ring.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_ in range(steps):
            ctx.kdk_step_batch(boxes, first, ngs, rss, rcs, st, params(s_, group, leaf, chunk),
                               ring)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # autotuning: one step per candidate (after one warm-up step), fastest wins
    tune = {}
    batch_run(1, 32, 16)
    for group in (16, 32, 64):
        for leaf in (8, 16, 32):
            tune[f"group {group} leaf {leaf}"] = (batch_run(1, group, leaf), group, leaf)
    best = min(tune.values())
    group, leaf = best[1], best[2]
    # PM tiles: deposit + interpolation kernel time over two steps per candidate chunk
    # (-1: no tiles)
    dep_tune = {}
    for chunk in (-1, 256, 1024, 4096):
        ctx.timing(enable=True, reset=True)
        batch_run(2, group, leaf, chunk)
        tk = ctx.timing(enable=False, reset=True)
        dep_tune[chunk] = (tk["pm_deposit"][0] + tk["pm_interp"][0]) / 2
    chunk = min(dep_tune, key=dep_tune.get)
    log(f"autotune: group {group}, leaf {leaf}, PM tile chunk {chunk}")
    batch_run(args.warmup, group, leaf, chunk)
    ctx.timing(enable=True, reset=True)
    ctx.pair_interactions(reset=True)
    t_batch = batch_run(K, group, leaf, chunk)
    kern = ctx.timing(enable=False, reset=True)
    pairs = ctx.pair_interactions(reset=True)
    final_eager = {k: getattr(st, k)[: st.n].clone() for k in ("x", "px", "gx")}

    # the same K steps as replays of one captured step (factors staged before each replay)
    log("graph capture and replays")
    copy_state(st, st0)
    ring.reset()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ctx.kdk_step_batch(boxes, first, ngs, rss, rcs, st, params(0, group, leaf, chunk), ring)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(K):
        ctx.kdk_step_batch_stage(params(s_, group, leaf, chunk))
        graph.replay()
        torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    ctx.check()
    graph_same = all(torch.equal(final_eager[k], getattr(st, k)[: st.n]) for k in final_eager)
    del graph
    ctx.close()

    # Run control: the lightcone keeps shrinking, so every box is coarsened again (R_lc = L/8);
    # the halt predicate compares the particle count with the last packing's and, once it has
    # fallen below 90%, the batch is packed again (new offsets, tables and context) and the
    # same steps are timed on the smaller batch.
    log("run control: second coarsening and re-packing")
    from paper_2005_05328_amd import ensemble
    rctx = dz.Context(max(first[b + 1] - first[b] for b in range(64)) + 64, max(ngs))
    cps = []
    for b in range(64):
        cp = dz.CoarsenParams()
        cp.R_lc, cp.b, cp.theta = 0.125 * specs[b]["L"], 0.0, 1.0
        cp.k_min = k_min_for(specs[b]["n_side"], 2 ** specs[b]["level"])
        cps.append(cp)
    counts, _ = ensemble.coarsen_boxes(rctx, boxes, st, first, cps)
    torch.cuda.synchronize()
    rctx.close()
    N2 = sum(counts)
    ratio, reasons = ensemble.control(counts, N, min_ratio=0.9)
    repack = {"particles_before": N, "particles_after": N2, "ratio": ratio,
              "halt_reasons": reasons, "repacked": False}
    if reasons & dz._abi.DZS_HALT_RATIO:
        pst, first2 = ensemble.repack(st, first, counts, capacity=N2 + 64)
        pctx = dz.Context(N2 + 64, side)
        pst0 = dz.State(N2 + 64)
        copy_state(pst0, pst)
        for s_ in range(args.warmup):
            pctx.kdk_step_batch(boxes, first2, ngs, rss, rcs, pst, params(s_, group, leaf, chunk), ring)
        copy_state(pst, pst0)
        ring.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_ in range(K):
            pctx.kdk_step_batch(boxes, first2, ngs, rss, rcs, pst, params(s_, group, leaf, chunk), ring)
        torch.cuda.synchronize()
        t_packed = time.perf_counter() - t0
        pctx.close()
        repack.update(repacked=True, ms_per_step_before=1e3 * t_batch / K,
                      ms_per_step_after=1e3 * t_packed / K)

    # the same steps box by box with the single-box call
    log("box-by-box comparison")
    bctx = dz.Context(max(first[b + 1] - first[b] for b in range(64)) + 64, max(ngs))
    states = []
    for b in range(64):
        lo, hi = first[b], first[b + 1]
        sub = _P()
        for k in ("x", "y", "z", "px", "py", "pz", "mult", "id", "type"):
            setattr(sub, k, getattr(allp, k)[lo:hi])
        states.append(dz.State.from_host(sub))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(K):
        for b in range(64):
            sp_ = params(s_, group, leaf, chunk)
            sp_.pm = dz.PMParams(ngs[b], prec, rss[b], 0, 0)
            sp_.tree = dz.TreeParams(rss[b], rcs[b], 0.5, leaf, group, prec, 0)
            bctx.kdk_step(boxes[b], states[b], sp_, ring)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    bctx.close()
    totals = {c: ms * calls for c, (ms, calls) in kern.items() if calls}
    avg_ms, calls = kern["tree_walk"]
    flops = FLOP_PER_INTERACTION * pairs / calls
    achieved = flops / (avg_ms * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if prec == dz.DZS_FP32 else PEAK_FP64_TFLOPS
    return {
        "metric": METRIC, "value": N * K / t_batch, "unit": UNIT, "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_batch / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == dz.DZS_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": (f"64-box ensemble (L 128-384 Mpc/h, 32^3-96^3 particles, "
                                f"meshes 64^3-192^3, Zel'dovich z=9, each coarsened once at "
                                f"level 1-3), {N} particles, {K} log KDK steps in one batched "
                                f"call per step"),
                   "preset": "c4", "particles": N, "boxes": 64, "parallelism": "1 GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None, "kernel": "tree_walk",
                     "avg_ms": avg_ms,
                     "work_per_launch": f"{pairs / calls:.4g} interactions x {FLOP_PER_INTERACTION} FLOP"},
        "cpu_baseline": None,
        "ensemble": {"batched_s": t_batch, "graph_replays_s": t_graph,
                     "graph_matches_eager_bitwise": bool(graph_same), "box_by_box_s": t_loop,
                     "batched_speedup": t_loop / t_batch, "graph_speedup": t_loop / t_graph,
                     "autotuned": {"group": group, "leaf": leaf, "tile_chunk": chunk},
                     "autotune_s_per_step": {k: v[0] for k, v in tune.items()},
                     "autotune_pm_tiles_ms": {str(k): v for k, v in dep_tune.items()},
                     "run_control": repack},
        "kernels_ms_per_step": {c: round(v / K, 4) for c, v in sorted(totals.items(),
                                                                    key=lambda kv: -kv[1])},
    }


HEADLINE_STATS_STEPS = 3   # steps after the timed ones with every kernel class timed
FULL_NSIDE = 64            # sky pixels of ~0.9 deg for the 1024^3 runs
LC_MESH = 128              # lightcone density mesh of the 1024^3 runs
MATCH_EVERY = 1024         # records of ids divisible by this are kept for the displacement match


def snapshot(st, torch):
    """Host copy (pageable) of the whole particle state."""
    n = st.n
    return {k: getattr(st, k)[:n].to("cpu") for k in st.F64 + ("mult", "id", "type")}, n


def restore(st, snap):
    arrays, n = snap
    for k, v in arrays.items():
        getattr(st, k)[:n].copy_(v)
    st.n = n


def cpu_baseline_sampled(W, ics, n_int=96):
    """The oracle timed on the host for a sample of the 1024^3 initial state, extrapolated to
    the whole box: its short-range sum (cell list, every source within r_cut) for the n_int^3
    lattice particles of a sub-cube, given the sources of that sub-cube grown by the cutoff
    plus one lattice cell; and its PM (deposit, FFT Poisson solve, 4-point gradient,
    interpolation) for a 1/4-per-side lattice subsample on a 1/4-per-side mesh, scaled to the
    full mesh by cells x log(cells) and to every particle."""
    import oracle
    oracle.build(force=False)
    n, L, lam = W["n_side"], W["L"], W["lam"]
    assert ics.max_disp < lam, "sources are taken by lattice index: displacements exceed a cell"
    box_o = oracle.Box(L=L, m0=W["m0"], eps0=W["eps0"])
    pad = int(math.ceil(W["r_cut"] / lam)) + 1
    side = n_int + 2 * pad
    c0 = n // 3   # sub-cube corner (lattice index), away from the periodic faces
    ax = np.arange(c0 - pad, c0 - pad + side) % n
    idx = ((ax[:, None, None] * n + ax[None, :, None]) * n + ax[None, None, :]).ravel()
    inner = np.zeros((side, side, side), bool)
    inner[pad:pad + n_int, pad:pad + n_int, pad:pad + n_int] = True
    targets = np.flatnonzero(inner.ravel())
    xs, ys, zs = ics.x[idx], ics.y[idx], ics.z[idx]
    ms = ics.mult[idx]
    t0 = time.perf_counter()
    oracle.short_range(xs, ys, zs, ms, box_o, W["r_s"], W["r_cut"], targets=targets)
    t_sr = time.perf_counter() - t0
    # PM on a subsample of every 4th lattice particle per side, mesh ng / 4
    f = 4
    sub = np.arange(0, n, f)
    sidx = ((sub[:, None, None] * n + sub[None, :, None]) * n + sub[None, None, :]).ravel()
    ng_s = W["ng"] // f
    m_s = W["m0"] * f ** 3
    box_s = oracle.Box(L=L, m0=m_s, eps0=W["eps0"] * f)
    t0 = time.perf_counter()
    oracle.pm_force(ics.x[sidx], ics.y[sidx], ics.z[sidx], ics.mult[sidx], box_s, ng_s,
                    W["r_s"])
    t_pm_s = time.perf_counter() - t0
    scale_pm = (f ** 3) * math.log(W["ng"] ** 3) / math.log(ng_s ** 3)
    N = W["N"]
    t_sr_full = t_sr / targets.size * N
    t_pm_full = t_pm_s * scale_pm
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh
                          if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": N / (t_sr_full + t_pm_full), "unit": UNIT, "cores": cores, "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(), "extrapolated": True,
            "sample": (f"extrapolated: the oracle's FP64 force on the {n}^3 initial state (z = 49). "
                       f"Short range (direct sum over every source within r_cut, cell list, "
                       f"OpenMP) for the {targets.size} particles of a {n_int}^3 lattice "
                       f"sub-cube: {t_sr:.1f} s, scaled to all {N} particles; PM (deposit, "
                       f"numpy FFT Poisson solve, 4-point gradient, interpolation) for a "
                       f"{n // f}^3 lattice subsample on a {ng_s}^3 mesh: {t_pm_s:.1f} s, scaled "
                       f"by {scale_pm:.1f} (cells x log cells) to the {W['ng']}^3 mesh; one force "
                       f"evaluation = {t_sr_full + t_pm_full:.3g} s"),
            "seconds": {"short_range_sample": t_sr, "pm_subsample": t_pm_s,
                        "short_range_extrapolated": t_sr_full, "pm_extrapolated": t_pm_full}}


class LightconeAccumulator:
    """Per-run lightcone products drained from the ring after every step (outside the step's
    timing): a CIC density mesh of the records, a sky map, the record count, and (id, offset)
    of the records whose id is divisible by MATCH_EVERY (for the twin displacement match)."""

    def __init__(self, torch, L, device="cuda"):
        self.torch, self.L = torch, L
        self.rho = torch.zeros(LC_MESH ** 3, dtype=torch.float64, device=device)
        self.sky = torch.zeros(12 * FULL_NSIDE ** 2, dtype=torch.float64, device=device)
        self.count = 0
        self.overflow = False
        self.ids, self.ds = [], []

    def drain(self, ring):
        from paper_2005_05328_amd import skymaps
        nrec = int(ring.count.item())
        self.overflow = self.overflow or bool(ring.overflow.item())
        if nrec:
            lightcone_density(ring, self.L, LC_MESH, self.rho)
            ids, mult, d = lightcone_records(ring)
            skymaps.sky_map(d, mult, FULL_NSIDE, self.sky)
            keep = (ids.to(self.torch.int64) % MATCH_EVERY) == 0
            self.ids.append(ids[keep].to(self.torch.int64))
            self.ds.append(d[keep].clone())
        self.count += min(nrec, ring.capacity)
        ring.reset()
        return nrec

    def fork(self):
        c = LightconeAccumulator.__new__(LightconeAccumulator)
        c.torch, c.L = self.torch, self.L
        c.rho, c.sky = self.rho.clone(), self.sky.clone()
        c.count, c.overflow = self.count, self.overflow
        c.ids, c.ds = list(self.ids), list(self.ds)
        return c


def compare_accumulated(a, b, L, eps0):
    """M-LC and the other lightcone diagnostics of two accumulated runs (b the reference);
    None with the reason when either run has no records."""
    torch = a.torch
    out = {"records": [a.count, b.count], "ring_overflow": [a.overflow, b.overflow]}
    if a.count == 0 or b.count == 0:
        out["no_records"] = [nm for nm, acc in (("dzs", a), ("std", b)) if acc.count == 0]
        out["M_LC_max_abs_P_ratio_minus_1"] = None
        return out
    rho_a, rho_b = a.rho.view(LC_MESH, LC_MESH, LC_MESH), b.rho.view(LC_MESH, LC_MESH, LC_MESH)
    k, pa, _ = power_spectrum(rho_a, L)
    _, pb, _ = power_spectrum(rho_b, L)
    ratio = pa / pb - 1.0
    from paper_2005_05328_amd import skymaps
    out["M_LC_max_abs_P_ratio_minus_1"] = float(np.abs(ratio).max())
    out["P_ratio_minus_1_by_bin"] = [round(float(v), 9) for v in ratio]
    out["k_bins_h_per_Mpc"] = [round(float(v), 5) for v in k]
    out["rms_pixel_density_difference"] = float(
        torch.sqrt(torch.mean((rho_a - rho_b) ** 2)) / rho_b.mean())
    out["sky_map"] = skymaps.compare_maps(a.sky.cpu().numpy(), b.sky.cpu().numpy(), FULL_NSIDE,
                                          SKY_LMAX)
    ia, da = torch.cat(a.ids), torch.cat(a.ds)
    ib, db = torch.cat(b.ids), torch.cat(b.ds)
    sa, oa = torch.sort(ia)
    sb, ob = torch.sort(ib)
    common = torch.isin(sa, sb)
    pos = torch.searchsorted(sb, sa[common])
    dx = da[oa[common]] - db[ob[pos]]
    dx = dx - L * torch.round(dx / L)
    r = (torch.sqrt((dx ** 2).sum(1)) / eps0).cpu().numpy()
    disp = {f"p{q}": float(np.percentile(r, q)) for q in (50, 99, 99.9)} if r.size else {}
    disp["max"] = float(r.max()) if r.size else None
    out["displacement_over_eps0"] = disp
    out["displacement_sample"] = (f"records with id divisible by {MATCH_EVERY}: {int(r.size)} "
                                  f"matched by id")
    out["displaced_fraction"] = ({f"over_{t}h": float((r > 2.8 * t).mean()) for t in (0.01, 0.1, 1, 8)}
                                 if r.size else {})
    return out


def run_headline(args, dz, torch, dzs_ics):
    """The 1024^3 configuration, both twins, in one process on one GPU.

    The DZS run and the full-resolution run are bitwise identical until the first step whose
    end boundary can merge (R_lc + b < sqrt(3)/2 L: the host check skips every earlier
    coarsening), so that shared prefix runs once and its wall time counts for both twins; the
    state is then copied to host memory, the DZS tail runs, the copy is restored and the
    full-resolution tail runs.  Every step is timed (wall clock, synchronised).

    value: particle force updates per second over the K timed steps (steps W+1 .. W+K of the
    schedule, after W warm-up steps), i.e. the particles forced in those steps over their wall
    time; only the tree walk carries HIP events in that region.  Three further steps time every
    kernel class (the breakdown).  M-W: whole-run wall time of the two twins.  M-LC and the sky
    maps: the lightcone records of each run, drained after every step.  M-F: the force alone on
    the final full-resolution state."""
    import copy
    P = dict(PRESETS["c5"])
    if args.n_side:
        f = args.n_side / P["n_side"]
        P.update(n_side=args.n_side, L=P["L"] * f, ng=int(round(P["ng"] * f)))
    W = workload(**P)
    W["tile_chunk"] = args.pm_chunk
    # groups of 64 in the FP32 walk: with each half of a dense group evaluated against the
    # entries near it, they are faster than 32 (256^3 walk: 21.8 against 22.7 ms at z = 49,
    # 28.6 against 30.5 ms on a Zel'dovich state at a = 0.3)
    W["group"] = args.group or FP32_GROUP
    W["leaf"] = args.leaf or W["leaf"]
    W["prec"] = dz.DZS_FP32
    N, L, n_steps = W["N"], W["L"], W["n_steps"]
    p_dzs = make_params(dz, W, True)
    p_std = make_params(dz, W, False)
    half_diag = 0.5 * math.sqrt(3.0) * L
    merging = [s for s, sp in enumerate(p_dzs)
               if sp.do_coarsen and sp.coarsen.R_lc + sp.coarsen.b < half_diag]
    prefix = merging[0] if merging else n_steps   # steps 0 .. prefix-1 are shared
    Wu = max(0, args.warmup)
    K = max(1, min(args.steps or 20, prefix - Wu - HEADLINE_STATS_STEPS))
    log(f"headline: N={N} L={L:g} ng={W['ng']} steps 1-{n_steps}; shared prefix 1-{prefix}; "
        f"warmup {Wu}, timed {Wu + 1}-{Wu + K}")
    t_job = time.perf_counter()
    t0 = time.perf_counter()
    ics = dzs_ics.zeldovich(W["n_side"], L, W["a_init"], seed=W["seed"], spectrum="bbks")
    log(f"initial conditions ready ({time.perf_counter() - t0:.0f} s)")
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        cpu = cpu_baseline_sampled(W, ics, n_int=max(8, min(128, W["n_side"] // 4)))
        log(f"cpu baseline (oracle, sampled): {cpu['value']:.3g} updates/s "
            f"({time.perf_counter() - t0:.0f} s)")
    box = dz.make_box(L, W["m0"], W["eps0"])
    ctx = dz.Context(N, W["ng"], fp32_meshes=True, no_copies=True)
    st = dz.State.from_host(ics)
    del ics
    # the initial force: a step with zero kicks and drift
    sp0 = copy.deepcopy(p_dzs[0])
    sp0.K1 = sp0.K2 = 0.0
    sp0.lc.D = 0.0
    sp0.do_lightcone = sp0.do_coarsen = 0
    ctx.kdk_step(box, st, sp0, None)
    torch.cuda.synchronize()
    ring = dz.LCRing(min(N, max(1 << 24, N // 5)))
    ring.reset()
    acc = LightconeAccumulator(torch, L)
    free, total = torch.cuda.mem_get_info()
    log(f"resident: {(total - free) / 2**30:.1f} GiB of {total / 2**30:.1f}")

    metrics = open(args.metrics, "w") if args.metrics else None

    def step(params, s_, acc_, run="shared"):
        t1 = time.perf_counter()
        rep = ctx.kdk_step(box, st, params[s_], ring)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        nrec = acc_.drain(ring)
        torch.cuda.synchronize()
        if metrics:
            metrics.write(json.dumps({"run": run, "step": s_ + 1, "a0": params[s_].lc.a0,
                                      "a1": params[s_].lc.a1, "wall_s": dt, "particles": st.n,
                                      "merged_nodes": int(rep.n_groups), "records": nrec}) + "\n")
            metrics.flush()
        return dt, int(rep.n_groups), nrec

    per_step = []          # shared prefix
    forced = []            # particles forced in each step
    # warm-up steps
    for s_ in range(Wu):
        per_step.append(step(p_dzs, s_, acc)[0])
        forced.append(st.n)
    # the timed steps: one synchronisation on each side, HIP events on the walk only
    ctx.timing(enable=True, reset=True, classes=("tree_walk",))
    ctx.pair_interactions(reset=True)
    torch.cuda.synchronize()
    t_timed0 = time.perf_counter()
    timed_forced = 0
    for s_ in range(Wu, Wu + K):
        dt, _, _ = step(p_dzs, s_, acc)
        per_step.append(dt)
        forced.append(st.n)
        timed_forced += st.n
        if (s_ + 1) % 5 == 0:
            log(f"  step {s_ + 1}: {dt:.3f} s")
    torch.cuda.synchronize()
    t_timed = time.perf_counter() - t_timed0
    walk = ctx.timing(enable=False, reset=True)
    pairs = ctx.pair_interactions(reset=True)
    walk_ms, walk_calls = walk["tree_walk"]
    # breakdown: every kernel class over the next steps
    ctx.timing(enable=True, reset=True)
    for s_ in range(Wu + K, Wu + K + HEADLINE_STATS_STEPS):
        per_step.append(step(p_dzs, s_, acc)[0])
        forced.append(st.n)
    kern = ctx.timing(enable=False, reset=True)
    stats_pairs = ctx.pair_interactions(reset=True)
    # the mesh kernels alone (inside a step they share the GPU with the tree build on the
    # other stream): three PM-only calls on the current state, then its force computed again
    # (same positions, same order: the same bits) for the next step's opening kick
    ctx.timing(enable=True, reset=True, classes=[c for c in HBM_CLASSES if c.startswith("pm_")])
    for _ in range(3):
        ctx.pm_force(box, st, sp0.pm)
    pm_alone = ctx.timing(enable=False, reset=True)
    ctx.kdk_step(box, st, sp0, None)
    torch.cuda.synchronize()
    for s_ in range(Wu + K + HEADLINE_STATS_STEPS, prefix):
        dt, _, _ = step(p_dzs, s_, acc)
        per_step.append(dt)
        forced.append(st.n)
        if (s_ + 1) % 10 == 0:
            log(f"  step {s_ + 1}: {dt:.3f} s")
    t_prefix = sum(per_step)
    log(f"shared prefix done: {t_prefix:.1f} s; copying the state to the host")
    t0 = time.perf_counter()
    snap = snapshot(st, torch)
    acc_std = acc.fork()
    log(f"  host copy {time.perf_counter() - t0:.1f} s")

    def tail(params, acc_, name):
        times, counts, merged = [], [], 0
        for s_ in range(prefix, n_steps):
            dt, m, nrec = step(params, s_, acc_, name)
            times.append(dt)
            counts.append(st.n)
            merged += m
            log(f"  {name} step {s_ + 1}: {dt:.3f} s, N = {st.n}, lightcone {nrec}")
        return times, counts, merged

    t_dzs_tail, n_dzs, merged_dzs = tail(p_dzs, acc, "dzs")
    mult_sum_dzs = int(st.mult[: st.n].to(torch.int64).sum().item())
    profile_dzs = mean_mass_by_distance(st, L)
    t0 = time.perf_counter()
    restore(st, snap)
    del snap
    torch.cuda.synchronize()
    log(f"  state restored ({time.perf_counter() - t0:.1f} s)")
    t_std_tail, n_std, merged_std = tail(p_std, acc_std, "std")
    lc = compare_accumulated(acc, acc_std, L, W["eps0"])
    # M-F: the force alone (keys, sort, tree build, PM, walk) on the final full-resolution state
    ctx.timing(enable=True, reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f_ms = []
    for r_ in range(4):
        e0.record()
        ctx.kdk_step(box, st, sp0, None)
        e1.record()
        torch.cuda.synchronize()
        if r_ > 0:
            f_ms.append(e0.elapsed_time(e1))
        else:
            ctx.timing(enable=True, reset=True)
    fk = ctx.timing(enable=False, reset=True)
    force_ms = float(np.median(f_ms))
    pm_ms = sum(fk[c][0] * fk[c][1] for c in fk if c.startswith("pm_")) / len(f_ms)
    tree_ms = sum(fk[c][0] * fk[c][1] for c in ("morton_keys", "radix_sort", "permute",
                                                "tree_build", "tree_moments", "tree_groups",
                                                "tree_walk") if c in fk) / len(f_ms)
    mf = {"M_F_force_updates_per_s": st.n / (force_ms * 1e-3), "force_ms": force_ms,
          "particles": st.n, "tree_ms": tree_ms, "tree_force_updates_per_s": st.n / (tree_ms * 1e-3),
          "pm_ms_on_second_stream": pm_ms,
          "method": ("median of 3 HIP-event-timed force evaluations after 1 warm-up (a step with "
                     "zero kick and drift factors: Morton keys, sort, tree build, PM, walk) on "
                     "the final full-resolution state (z = 0); tree_ms: the tree kernel classes' "
                     "time (the PM overlaps them on a second stream)")}
    free, total = torch.cuda.mem_get_info()
    ctx.close()
    if metrics:
        metrics.close()
    t_dzs = t_prefix + sum(t_dzs_tail)
    t_std = t_prefix + sum(t_std_tail)
    fp32 = True
    Cc = W["ng"] ** 3
    totals = {c: ms * calls for c, (ms, calls) in kern.items() if calls}
    flops = FLOP_PER_INTERACTION * pairs / walk_calls
    achieved = flops / (walk_ms * 1e-3) / 1e12
    hbm = {}
    for cls in HBM_CLASSES:
        src = pm_alone if cls.startswith("pm_") else kern
        if cls not in src or not src[cls][1]:
            continue
        ms = src[cls][0]
        b = algorithmic_bytes(cls, N, Cc, fp32)
        hbm[cls] = {"avg_ms": ms, "achieved_GBps": b / (ms * 1e-3) / 1e9,
                    "frac": b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                    "timed": ("alone: three PM calls on the state after the timed steps"
                              if cls.startswith("pm_") else "in the breakdown steps")}
    twin = {
        "kind": "DZS vs full resolution, whole 100-step runs",
        "M_W_dzs_over_std": t_dzs / t_std, "dzs_s": t_dzs, "std_s": t_std,
        "shared_prefix": (f"steps 1-{prefix} (no node can merge before the boundary after step "
                          f"{prefix + 1}: R_lc + b >= sqrt(3)/2 L) run once, {t_prefix:.1f} s, "
                          f"counted in both"),
        "tail_s": {"dzs": sum(t_dzs_tail), "std": sum(t_std_tail)},
        "tail_per_step_s": {"dzs": [round(v, 3) for v in t_dzs_tail],
                            "std": [round(v, 3) for v in t_std_tail]},
        "particles_after_tail_steps": {"dzs": n_dzs, "std": n_std},
        "merged_nodes": [merged_dzs, merged_std],
        "summed_multiplicity_conserved": mult_sum_dzs == N,
        "mean_mass_by_distance_dzs": profile_dzs,
        "lightcone": lc,
        "paper": ("T_DZS/T_STD 0.60-0.64 for the paper's fiducial DZS on its 8192 Mpc/h, 512^3 run "
                  "(Table particle_gain_all, CPU, hardware unstated)"),
    }
    out = {
        "metric": METRIC, "value": timed_forced / t_timed, "unit": UNIT, "n_gpus": 1, "steps": K,
        "warmup": Wu, "ms_per_step": 1e3 * t_timed / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{W['n_side']}^3 particles (1 GPU), L={L:g} Mpc/h, mesh "
                                f"{W['ng']}^3, Zel'dovich z=49 BBKS seed {W['seed']}, 100 log KDK "
                                f"steps to z=0, DZS 2x2x2 then 4x4x4 (l_max 4 lambda, theta 0.1, "
                                f"b 5 lambda) + lightcone output, tree theta {W['theta_tree']}, "
                                f"precision form (FP32 pair/mesh/FFT, FP64 state); timed: steps "
                                f"{Wu + 1}-{Wu + K} (full resolution, z = "
                                f"{1 / p_dzs[Wu].lc.a0 - 1:.1f} to {1 / p_dzs[Wu + K - 1].lc.a1 - 1:.1f})"),
                   "preset": "c5", "particles": N, "mesh": W["ng"], "box": L,
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     # the committed counters cover this exact run: 1024^3, default group and
                     # leaf sizes, the launches of steps 6-25
                     "traffic": (headline_walk_traffic() if not (args.n_side or args.group or
                                 args.leaf) and (Wu, K) == (5, 20) else None),
                     "traffic_unit": "bytes per launch",
                     "kernel": "tree_walk", "avg_ms": walk_ms,
                     "work_per_launch": f"{pairs / walk_calls:.4g} interactions x {FLOP_PER_INTERACTION} FLOP",
                     "timed_on": "the walk's own stream, HIP events around each launch in the timed steps"},
        "cpu_baseline": cpu, "twin": twin, "force_rate": mf, "hbm_kernels": hbm,
        "pair_interactions_per_step": pairs / K,
        "kernels_ms_per_step": {c: round(v / HEADLINE_STATS_STEPS, 3) for c, v in
                                sorted(totals.items(), key=lambda kv: -kv[1])},
        "kernels_note": (f"every kernel class over steps {Wu + K + 1}-{Wu + K + HEADLINE_STATS_STEPS} "
                         f"(after the timed ones); the mesh solve runs on a second stream, so "
                         f"the classes overlap"),
        "memory": {"device_used_GiB": (total - free) / 2 ** 30, "device_total_GiB": total / 2 ** 30},
        "job_s": time.perf_counter() - t_job,
    }
    return out


SWEEP = {  # parameter -> values; the fiducial setting is theta 0.1, b 5 lambda, l_max 4 lambda
    "theta": (0.01, 0.03, 0.1, 0.2, 0.5, 1.0),
    "alpha_dyn": (1e-4, 1e-3, 1e-2, 1e-1),
    "b_over_lambda": (100.0, 10.0, 5.0, 2.0, 1.0, 0.0),
    "lmax_over_lambda": (2, 4, 8, 32, 64),
}


def run_sweep(args, dz, torch, dzs_ics):
    """The de-refinement parameters one at a time around the fiducial setting, on a small
    box with the lightcone geometry of a large one: 128^3 particles, L = 8192 Mpc/h (64 Mpc/h
    per particle), mesh 256^3, 100 log steps from z = 49 in the precision form; DZS starts
    once R_lc + b < sqrt(3)/2 L (step 37).  Each run starts from the same initial state and
    force; reported: N_fin / N_init, wall time against the full-resolution run, and the
    lightcone comparison against it (64^3 density mesh of the records, drained every step)."""
    import copy
    W = workload(n_side=128, L=8192.0, ng=256, seed=20050540, n_steps=100, lmax_over_lambda=4)
    W["prec"] = dz.DZS_FP32
    N, lam = W["N"], W["lam"]
    ics = dzs_ics.zeldovich(W["n_side"], W["L"], W["a_init"], seed=W["seed"], spectrum="bbks")
    box = dz.make_box(W["L"], W["m0"], W["eps0"])
    ctx = dz.Context(N, W["ng"])
    st0 = dz.State.from_host(ics)
    base = make_params(dz, W, True)
    sp0 = copy.deepcopy(base[0])
    sp0.K1 = sp0.K2 = 0.0
    sp0.lc.D = 0.0
    sp0.do_lightcone = sp0.do_coarsen = 0
    ctx.kdk_step(box, st0, sp0, None)
    st = dz.State(N)
    ring = dz.LCRing(N)
    M = 64

    def one(theta=0.1, alpha=None, b=5.0, lmax=4, dzs=True):
        params = make_params(dz, W, dzs)
        for sp in params:
            sp.coarsen.b = b * lam
            sp.coarsen.k_min = k_min_for(W["n_side"], lmax)
            if alpha is None:
                sp.coarsen.theta = theta
            else:
                sp.coarsen.criterion = dz.DZS_CRIT_DYNAMICAL
                sp.coarsen.alpha_dyn = alpha
        copy_state(st, st0)
        rho = torch.zeros(M ** 3, dtype=torch.float64, device="cuda")
        ring.reset()
        torch.cuda.synchronize()
        wall = 0.0
        for sp in params:
            t1 = time.perf_counter()
            ctx.kdk_step(box, st, sp, ring)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t1
            lightcone_density(ring, W["L"], M, rho)
            ring.reset()
            torch.cuda.synchronize()
        return wall, st.n, rho.view(M, M, M)

    one(dzs=False)   # warm-up of every kernel and allocation
    t_std, _, rho_std = one(dzs=False)
    k, p_std, _ = power_spectrum(rho_std, W["L"])
    rows = []
    for name, values in SWEEP.items():
        for v in values:
            kw = {"theta": dict(theta=v), "alpha_dyn": dict(alpha=v),
                  "b_over_lambda": dict(b=v), "lmax_over_lambda": dict(lmax=v)}[name]
            wall, n_fin, rho = one(**kw)
            _, p, _ = power_spectrum(rho, W["L"])
            rows.append({"parameter": name, "value": v, "n_fin_over_n_init": n_fin / N,
                         "t_dzs_over_t_std": wall / t_std,
                         "M_LC_max_abs_P_ratio_minus_1": float(np.abs(p / p_std - 1.0).max()),
                         "rms_pixel_density_difference":
                             float(torch.sqrt(torch.mean((rho - rho_std) ** 2)) / rho_std.mean())})
            log(f"  {name} = {v}: N_fin/N_init {n_fin / N:.4f}, T/T_std {wall / t_std:.4f}")
    ctx.close()
    return {"sweep": "DZS parameters, one at a time around theta 0.1, b 5 lambda, l_max 4 lambda",
            "workload": f"128^3 particles, L=8192 Mpc/h, mesh 256^3, Zel'dovich z=49 BBKS seed "
                        f"{W['seed']}, 100 log KDK steps, lightcone, tree theta 0.5, precision form",
            "std_wall_s": t_std, "rows": rows}


def _smooth(n):
    while n % 2 == 0:
        n //= 2
    while n % 3 == 0:
        n //= 3
    return n == 1


FP32_GROUP = 64   # targets per walk group of the FP32 runs (the FP64 walk keeps 32)


def workload(n_side=128, L=256.0, ng=256, seed=20050529, n_steps=50, lmax_over_lambda=2,
             leaf=16, **_):
    import dzs_ics
    lam = L / n_side
    return dict(n_side=n_side, N=n_side ** 3, L=L, ng=ng, r_s=1.25 * L / ng,
                r_cut=4.5 * 1.25 * L / ng, eps0=lam / 40, m0=dzs_ics.particle_mass(L, n_side ** 3),
                lam=lam, a_init=1.0 / 50.0, n_steps=n_steps, theta_tree=0.5, theta_dzs=0.1,
                b=5 * lam, lmax_over_lambda=lmax_over_lambda, seed=seed, leaf=leaf, group=32)


def k_min_for(n_side, j):
    k = 0
    while n_side > j * (1 << k):
        k += 1
    return k


def make_params(dz, W, do_coarsen):
    a = np.exp(np.linspace(math.log(W["a_init"]), 0.0, W["n_steps"] + 1))
    out = []
    for s in range(W["n_steps"]):
        sp = dz.step_factors(float(a[s]), float(a[s + 1]), 0.3)
        sp.do_lightcone = 1
        # DZS acts at a step boundary only when another step follows it
        sp.do_coarsen = 1 if (do_coarsen and s + 1 < W["n_steps"]) else 0
        sp.coarsen.R_lc = math.sqrt(sp.lc.chi2_1)
        sp.coarsen.b = W["b"]
        sp.coarsen.theta = W["theta_dzs"]
        sp.coarsen.k_min = k_min_for(W["n_side"], W["lmax_over_lambda"])
        sp.pm = dz.PMParams(W["ng"], W["prec"], W["r_s"], 0, W.get("tile_chunk", 0))
        sp.tree = dz.TreeParams(W["r_s"], W["r_cut"], W["theta_tree"], W["leaf"], W["group"],
                                W["prec"], 0)
        out.append(sp)
    return out


def copy_state(dst, src):
    for k in src.F64 + ("mult", "id", "type"):
        getattr(dst, k).copy_(getattr(src, k))
    dst.n = src.n


# algorithmic bytes moved per launch, by kernel class (N particles, C mesh cells); in the
# precision form mesh values are 4-byte reals / 8-byte complex instead of 8 / 16
def algorithmic_bytes(cls, N, C, fp32=False):
    r, c = (4, 8) if fp32 else (8, 16)
    n = round(C ** (1.0 / 3.0))
    H = (n // 2 + 1) * n * n  # complex cells of the half spectrum (k_x = 0 .. n/2)
    return {
        "kick": 72 * N, "drift_lightcone": 72 * N, "morton_keys": 36 * N,
        "pm_deposit": 28 * N + 8 * C,
        # x pass: forward reads the 8-byte fixed-point mesh and writes the half spectrum;
        # inverse reads it and writes the real potential (the class averages both launches)
        "pm_fft_x": ((8 * C + c * H) + (c * H + r * C)) // 2,
        "pm_fft_y": 2 * c * H, "pm_fft_z_green": 2 * c * H,
        "pm_interp": 48 * N + r * C,
    }.get(cls)


HBM_CLASSES = ("pm_deposit", "pm_fft_x", "pm_fft_y", "pm_fft_z_green", "pm_interp", "kick",
               "drift_lightcone")
TRAFFIC_SOURCES = {"tree_walk": "tree.hip", "kick": "particles.hip",
                   "drift_lightcone": "particles.hip"}


def measured_traffic(prec_name, workload_is_default):
    """Counter-measured HBM bytes per launch from the committed rocprofv3 summary, by kernel
    class, for the default 128^3 workload only; a class whose sources changed since the
    counters were taken gets None."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_128cube.md")
    if not workload_is_default or not os.path.exists(path):
        return {}
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return {}
    doc = json.loads(m.group(1))
    csrc = os.path.join(ROOT, "paper_2005_05328_amd", "csrc")

    def same(f):
        h = hashlib.sha256(open(os.path.join(csrc, f), "rb").read()).hexdigest()[:16]
        return doc["source_sha256_16"].get(f) == h
    out = {}
    for cls, b in doc["bytes_per_launch"].get(prec_name, {}).items():
        src = TRAFFIC_SOURCES.get(cls, "pm.hip")
        out[cls] = b if (same(src) and same("internal.h")) else None
    return out


def headline_walk_traffic():
    """The walk's counter-measured HBM bytes per launch at the 1024^3 headline (FETCH_SIZE +
    WRITE_SIZE over the timed steps' launches, scaled by a plain copy) from the committed
    rocprofv3 summary; None when it is missing or the walk's sources changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_1024cube_walk.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    doc = json.loads(m.group(1))
    csrc = os.path.join(ROOT, "paper_2005_05328_amd", "csrc")
    for f, h in doc["source_sha256_16"].items():
        if hashlib.sha256(open(os.path.join(csrc, f), "rb").read()).hexdigest()[:16] != h:
            return None
    return doc["bytes_per_launch"]


def cpu_baseline(W, ics, box_o, n_steps=8):
    """The oracle timed on the host: its kick-drift-kick step (FP64 PM on the full mesh plus
    the direct-sum short range for every particle, lightcone test) over the first n_steps
    steps of the same schedule, on all particles."""
    import oracle
    oracle.build(force=False)
    a = np.exp(np.linspace(math.log(W["a_init"]), 0.0, W["n_steps"] + 1))
    g = oracle.total_force(ics.x, ics.y, ics.z, ics.mult, box_o, W["ng"], W["r_s"], W["r_cut"])
    ps = ics
    t0 = time.perf_counter()
    for s in range(n_steps):
        fac = oracle.step_factors(float(a[s]), float(a[s + 1]))
        fac.update(a0=float(a[s]), a1=float(a[s + 1]))
        ps, g, _, _ = oracle.kdk_step(ps, g, box_o, fac, W["ng"], W["r_s"], W["r_cut"],
                                      [0.0, 0.0, 0.0])
    t = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         None)
    except OSError:
        pass
    return {"value": W["N"] * n_steps / t, "unit": UNIT, "cores": cores, "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": (f"the oracle's FP64 kick-drift-kick step (full PM {W['ng']}^3, direct-sum "
                       f"short range for all {W['N']} particles, lightcone test) over the first "
                       f"{n_steps} of the {W['n_steps']} steps (z = 49 to "
                       f"{1 / a[n_steps] - 1:.1f}), {t:.1f} s; OpenMP short range, "
                       f"single-threaded numpy FFT; the GPU figure averages all timed steps")}


def force_rate(ctx, box, st, W, dz, torch, reps=10, warm=3):
    """M-F: particle force updates per second of one full force evaluation (PM, then the
    tree: keys, sort, build, walk) on the current state, median of `reps` HIP-event-timed
    calls after `warm` warm-ups; also the tree-only and PM-only times."""
    pm = dz.PMParams(W["ng"], W["prec"], W["r_s"], 0, W.get("tile_chunk", 0))
    tp = dz.TreeParams(W["r_s"], W["r_cut"], W["theta_tree"], W["leaf"], W["group"], W["prec"], 1)

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    calls = {"force": lambda: (ctx.pm_force(box, st, pm), ctx.tree_force(box, st, tp)),
             "pm": lambda: ctx.pm_force(box, st, pm),
             "tree": lambda: ctx.tree_force(box, st, tp)}
    med = {}
    for name, fn in calls.items():
        for _ in range(warm):
            fn()
        med[name] = float(np.median([timed(fn) for _ in range(reps)]))
    n = st.n
    return {"M_F_force_updates_per_s": n / (med["force"] * 1e-3), "force_ms": med["force"],
            "tree_force_updates_per_s": n / (med["tree"] * 1e-3), "tree_force_ms": med["tree"],
            "pm_force_ms": med["pm"], "particles": n,
            "method": f"median of {reps} after {warm} warm-ups, HIP events, final state"}


# ---- twin-run diagnostics (measurement only: they run after the timed region) -------------

def lightcone_records(ring):
    """Device views of the records in a ring: ids, multiplicities, offsets d (n x 3)."""
    import torch
    n = min(int(ring.count.item()), ring.capacity)
    rec = ring.buf[: 8 * n].view(n, 8)
    ints = rec.view(torch.int32)[:, :2]
    return ints[:, 0], ints[:, 1].to(torch.float64), rec[:, 2:5]


def lightcone_density(ring, L, M, rho=None):
    """Mass (in particle masses) of the lightcone records deposited by cloud-in-cell onto an
    M^3 mesh, each record at its crossing position wrapped into the box (observer at 0);
    added to `rho` (flat, M^3) when given."""
    import torch
    _, mult, d = lightcone_records(ring)
    u = torch.remainder(d, L) * (M / L)
    i0 = torch.floor(u)
    f = u - i0
    i0 = i0.to(torch.int64) % M
    if rho is None:
        rho = torch.zeros(M ** 3, dtype=torch.float64, device=d.device)
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1 - f[:, 0]
        ix = (i0[:, 0] + cx) % M
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1 - f[:, 1]
            iy = (i0[:, 1] + cy) % M
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1 - f[:, 2]
                iz = (i0[:, 2] + cz) % M
                rho.index_add_(0, (ix * M + iy) * M + iz, mult * wx * wy * wz)
    return rho.view(M, M, M)


def power_spectrum(rho, L, n_bins=16):
    """P(k) of the density contrast in logarithmic bins from the fundamental mode to half
    the Nyquist frequency (bin centres, power, mode counts)."""
    import torch
    M = rho.shape[0]
    delta = rho / rho.mean() - 1.0
    dk = torch.fft.rfftn(delta)
    pk = (dk.real ** 2 + dk.imag ** 2) * (L ** 3 / M ** 6)
    kf = 2 * math.pi / L
    n1 = torch.fft.fftfreq(M, 1.0 / M, device=rho.device, dtype=torch.float64)
    n3 = torch.fft.rfftfreq(M, 1.0 / M, device=rho.device, dtype=torch.float64)
    kk = kf * torch.sqrt(n1[:, None, None] ** 2 + n1[None, :, None] ** 2 + n3[None, None, :] ** 2)
    edges = torch.logspace(math.log10(kf), math.log10(kf * M / 4), n_bins + 1,
                           dtype=torch.float64, device=rho.device)
    idx = torch.bucketize(kk.flatten(), edges) - 1
    ok = (idx >= 0) & (idx < n_bins) & (kk.flatten() > 0)
    p = torch.zeros(n_bins, dtype=torch.float64, device=rho.device)
    c = torch.zeros(n_bins, dtype=torch.float64, device=rho.device)
    p.index_add_(0, idx[ok], pk.flatten()[ok])
    c.index_add_(0, idx[ok], torch.ones_like(pk.flatten()[ok]))
    keep = c > 0
    kc = torch.sqrt(edges[:-1] * edges[1:])
    return kc[keep].cpu().numpy(), (p[keep] / c[keep]).cpu().numpy(), c[keep].cpu().numpy()


SKY_NSIDE, SKY_LMAX = 32, 48   # equal-area sky pixels of ~1.8 deg, C_l to l = 48


def mean_mass_by_distance(st, L, x_obs=(0.0, 0.0, 0.0), n_bins=16):
    """Mean multiplicity of the particles in shells of minimum-image distance from the
    observer (the paper's mean particle mass against d_obs), out to sqrt(3)/2 L."""
    import torch
    n = st.n
    d2 = torch.zeros(n, dtype=torch.float64, device=st.x.device)
    for k, xo in zip(("x", "y", "z"), x_obs):
        dd = getattr(st, k)[:n] - xo
        dd = dd - L * torch.floor(dd / L + 0.5)
        d2 += dd * dd
    edges = np.linspace(0.0, 0.5 * math.sqrt(3.0) * L, n_bins + 1)
    idx = torch.clamp((torch.sqrt(d2) / edges[1]).to(torch.int64), 0, n_bins - 1)
    mult = st.mult[:n].to(torch.float64)
    cnt = torch.zeros(n_bins, dtype=torch.float64, device=d2.device).index_add_(
        0, idx, torch.ones_like(mult))
    mass = torch.zeros(n_bins, dtype=torch.float64, device=d2.device).index_add_(0, idx, mult)
    c, m = cnt.cpu().numpy(), mass.cpu().numpy()
    return {"shell_outer_radius": [round(float(v), 3) for v in edges[1:]],
            "mean_multiplicity": [round(float(a / b), 4) if b else None for a, b in zip(m, c)]}


def compare_lightcones(ring_a, rho_a, ring_b, rho_b, L, eps0):
    """M-LC (max |P_a/P_b - 1| over the bins), rms pixel density difference, and the
    displacement percentiles of records present in both runs, in units of eps0."""
    import torch
    k, pa, _ = power_spectrum(rho_a, L)
    _, pb, _ = power_spectrum(rho_b, L)
    ratio = pa / pb - 1.0
    rms = float(torch.sqrt(torch.mean((rho_a - rho_b) ** 2)) / rho_b.mean())
    ia, _, da = lightcone_records(ring_a)
    ib, _, db = lightcone_records(ring_b)
    sa, oa = torch.sort(ia.to(torch.int64))
    sb, ob = torch.sort(ib.to(torch.int64))
    common = torch.isin(sa, sb)
    pos = torch.searchsorted(sb, sa[common])
    dx = da[oa[common]] - db[ob[pos]]
    dx = dx - L * torch.round(dx / L)
    r = (torch.sqrt((dx ** 2).sum(1)) / eps0).cpu().numpy()
    pct = {f"p{q}": float(np.percentile(r, q)) for q in (50, 99, 99.9)} if r.size else {}
    pct["max"] = float(r.max()) if r.size else None
    # the paper's accuracy statements use the softening length h = 2.8 eps
    frac_h = ({f"over_{t}h": float((r > 2.8 * t).mean()) for t in (0.01, 0.1, 1, 8)}
              if r.size else {})
    from paper_2005_05328_amd import skymaps
    _, ma, _ = lightcone_records(ring_a)
    _, mb, _ = lightcone_records(ring_b)
    sky_a = skymaps.sky_map(da, ma, SKY_NSIDE)
    sky_b = skymaps.sky_map(db, mb, SKY_NSIDE)
    sky = skymaps.compare_maps(sky_a.cpu().numpy(), sky_b.cpu().numpy(), SKY_NSIDE, SKY_LMAX)
    return {"M_LC_max_abs_P_ratio_minus_1": float(np.abs(ratio).max()),
            "sky_map": sky, "displaced_fraction": frac_h,
            "P_ratio_minus_1_by_bin": [round(float(v), 8) for v in ratio],
            "k_bins_h_per_Mpc": [round(float(v), 5) for v in k],
            "rms_pixel_density_difference": rms,
            "records": [int(ia.numel()), int(ib.numel())], "records_matched": int(r.size),
            "displacement_over_eps0": pct}


def force_error(g, ref):
    """rms relative error over particles and the 99th percentile of the per-particle
    relative error |g - ref| / |ref|."""
    import torch
    e = torch.sqrt(((g - ref) ** 2).sum(0))
    m = torch.sqrt((ref ** 2).sum(0))
    rms = float(torch.sqrt((e ** 2).mean() / (m ** 2).mean()))
    rel = (e / torch.clamp(m, min=1e-300)).cpu().numpy()
    return {"rms_rel": rms, "p99_rel": float(np.percentile(rel, 99)),
            "max_rel": float(rel.max())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(PRESETS) + ["sweep"], default="c5")
    ap.add_argument("--steps", type=int, default=0,
                    help="timed steps (default: 20 for c5, the whole run otherwise)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-side", type=int, default=0,
                    help="particles per side (box and mesh scaled with it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-twin", action="store_true")
    ap.add_argument("--no-force-rate", action="store_true",
                    help="skip the force-only rate (M-F) measured after the run")
    ap.add_argument("--group", type=int, default=0, help="targets per wave group (power of 2)")
    ap.add_argument("--leaf", type=int, default=0, help="particles per tree leaf")
    ap.add_argument("--pm-chunk", type=int, default=0,
                    help="particles per LDS tile of deposit and interpolation (0: default, -1: none)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (the reference "
                         "for scaling HBM byte counters), then exit")
    ap.add_argument("--hier", type=int, default=0, metavar="B",
                    help="individual power-of-two time steps: 2^B sub-steps per global step")
    ap.add_argument("--pm-global", action="store_true",
                    help="with --hier: the long-range force on the global step only (the tree "
                         "built once per global step and refreshed at every sub-step)")
    ap.add_argument("--eta", type=float, default=0.025,
                    help="accuracy parameter of the individual time-step bins")
    ap.add_argument("--metrics", default=None, metavar="JSONL",
                    help="c5: one JSON line per step (run, step, a0, a1, wall_s, particles, "
                         "merged_nodes, records) written to this file as the run goes")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default=None,
                    help="fp64: plain form; fp32: FP32 pair, mesh and FFT arithmetic "
                         "(default: the workload's)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "copies": 3}), flush=True)
        return
    sys.path.insert(0, ROOT)
    import dzs_ics
    import paper_2005_05328_amd as dz

    if args.workload == "c4":
        print(json.dumps(run_ensemble(args, dz, torch, dzs_ics)), flush=True)
        return
    if args.workload == "sweep":
        print(json.dumps(run_sweep(args, dz, torch, dzs_ics)), flush=True)
        return
    if args.workload == "c5":
        print(json.dumps(run_headline(args, dz, torch, dzs_ics)), flush=True)
        return
    P = dict(PRESETS[args.workload])
    if args.n_side:
        f = args.n_side / P["n_side"]
        P.update(n_side=args.n_side, L=P["L"] * f, ng=int(round(P["ng"] * f)))
    W = workload(**P)
    if args.group:
        W["group"] = args.group
    if args.leaf:
        W["leaf"] = args.leaf
    W["tile_chunk"] = args.pm_chunk
    prec_name = args.precision or P["precision"]
    W["prec"] = dz.DZS_FP32 if prec_name == "fp32" else dz.DZS_FP64
    fp32 = W["prec"] == dz.DZS_FP32
    twin_kind = None if args.no_twin else P["twin"]
    if not args.group and fp32 and twin_kind != "precision":
        W["group"] = FP32_GROUP   # an FP32 run without an FP64 twin
    K = max(1, min(args.steps or W["n_steps"], W["n_steps"]))
    log(f"workload {args.workload}: N={W['N']} L={W['L']} ng={W['ng']} {prec_name} steps={K} "
        f"warmup={args.warmup} twin={twin_kind}")
    ics = dzs_ics.zeldovich(W["n_side"], W["L"], W["a_init"], seed=W["seed"], spectrum="bbks")
    log("initial conditions ready")
    box = dz.make_box(W["L"], W["m0"], W["eps0"])
    ctx = dz.Context(W["N"], W["ng"], hier_split=args.pm_global)
    st0 = dz.State.from_host(ics)

    def force(state, prec):
        ctx.pm_force(box, state,
                     dz.PMParams(W["ng"], prec, W["r_s"], 0, W.get("tile_chunk", 0)))
        ctx.tree_force(box, state, dz.TreeParams(W["r_s"], W["r_cut"], W["theta_tree"],
                                                 W["leaf"], W["group"], prec, 1))
        torch.cuda.synchronize()
        return torch.stack([state.gx[: state.n], state.gy[: state.n], state.gz[: state.n]]).clone()

    g0 = force(st0, W["prec"])
    twin_prec = W["prec"]
    if twin_kind == "precision":
        twin_prec = dz.DZS_FP64
    g0_twin = force(st0, twin_prec) if twin_prec != W["prec"] else g0
    ic_force_error = force_error(g0, g0_twin) if twin_kind == "precision" else None
    params_main = make_params(dz, W, True)
    W_twin = dict(W, prec=twin_prec)
    params_twin = make_params(dz, W_twin, twin_kind != "dzs")
    st = dz.State(W["N"])
    ring = dz.LCRing(W["N"])
    ring_twin = dz.LCRing(W["N"]) if twin_kind else None

    def run(params, steps, timed, g_init, rg):
        copy_state(st, st0)
        for a_, k in enumerate(("gx", "gy", "gz")):
            getattr(st, k)[: st0.n].copy_(g_init[a_])
        rg.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        merged = 0
        for s_ in range(steps):
            if args.hier:
                # individual power-of-two steps inside the global step, limiter at R_lc + b
                sp_ = params[s_]
                rep = ctx.kdk_step_hier(box, st, sp_, args.hier, args.eta, sp_.lc.a0, sp_.lc.a1,
                                        limiter=True,
                                        R_lim=math.sqrt(sp_.lc.chi2_0) + sp_.coarsen.b, ring=rg,
                                        pm_global=args.pm_global)
            else:
                rep = ctx.kdk_step(box, st, params[s_], rg)
            merged += int(rep.n_groups)
            if timed and (s_ + 1) % 10 == 0:
                log(f"  step {s_ + 1}/{steps}")
        torch.cuda.synchronize()
        return time.perf_counter() - t0, merged

    log("warmup")
    run(params_main, args.warmup, False, g0, ring)
    log("timed run")
    ctx.timing(enable=True, reset=True)
    ctx.pair_interactions(reset=True)
    t_main, merged = run(params_main, K, True, g0, ring)
    kern = ctx.timing(enable=False, reset=True)
    pairs = ctx.pair_interactions(reset=True)
    n_records = int(ring.count.item())
    n_final = st.n
    M = min(W["ng"], 256)
    twin = None
    if twin_kind:
        final_main = {k: getattr(st, k)[: st.n].clone() for k in ("x", "y", "z", "px", "py", "pz")}
        mass_profile = mean_mass_by_distance(st, W["L"])
        rho_main = lightcone_density(ring, W["L"], M)
        log(f"timed twin ({'full resolution' if twin_kind == 'dzs' else 'FP64 plain form'})")
        t_twin, merged_twin = run(params_twin, K, True, g0_twin, ring_twin)
        rho_twin = lightcone_density(ring_twin, W["L"], M)
        lc = compare_lightcones(ring, rho_main, ring_twin, rho_twin, W["L"], W["eps0"])
        if twin_kind == "dzs":
            same = n_final == st.n and all(torch.equal(final_main[k], getattr(st, k)[: st.n])
                                           for k in final_main)
            twin = {"kind": "DZS vs full resolution", "std_s": t_twin, "dzs_s": t_main,
                    "dzs_over_std": t_main / t_twin, "twins_bitwise_identical": bool(same),
                    "merged_nodes": merged, "particles_final": [n_final, st.n],
                    "mean_mass_by_distance": mass_profile, "lightcone": lc}
        else:
            del final_main
            log("forces on the final plain-form state in both forms")
            g64 = force(st, dz.DZS_FP64)
            g32 = force(st, dz.DZS_FP32)
            twin = {"kind": "precision form vs FP64 plain form", "precision_s": t_main,
                    "plain_s": t_twin, "precision_over_plain": t_main / t_twin,
                    "merged_nodes": [merged, merged_twin],
                    "force_error_initial": ic_force_error,
                    "force_error_final_state": force_error(g32, g64),
                    "lightcone": lc}

    N, C = W["N"], W["ng"] ** 3
    totals = {c: ms * calls for c, (ms, calls) in kern.items() if calls}
    dom = max(totals, key=totals.get)
    avg_ms, calls = kern[dom]
    default = (args.workload == "c2" and not args.n_side and K == 50 and args.warmup == 2
               and not args.group and not args.leaf)
    traffic = measured_traffic(prec_name, default)
    if dom == "tree_walk":
        flops = FLOP_PER_INTERACTION * pairs / calls
        achieved = flops / (avg_ms * 1e-3) / 1e12
        peak = PEAK_FP32_TFLOPS if fp32 else PEAK_FP64_TFLOPS
        roofline = {"bound": "alu", "achieved": achieved, "peak": peak,
                    "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic.get(dom),
                    "kernel": dom, "avg_ms": avg_ms,
                    "work_per_launch": f"{pairs / calls:.4g} interactions x {FLOP_PER_INTERACTION} FLOP"}
    else:
        b = algorithmic_bytes(dom, N, C, fp32)
        achieved = (b / (avg_ms * 1e-3) / 1e9) if b else None
        roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM_GBS if achieved else None,
                    "traffic": traffic.get(dom), "kernel": dom, "avg_ms": avg_ms}
    # the HBM-bound kernels beside it: algorithmic GB/s against the 8 TB/s peak, and the
    # counter-measured bytes where available
    hbm = {}
    for cls in HBM_CLASSES:
        if cls not in kern or not kern[cls][1]:
            continue
        ms = kern[cls][0]
        b = algorithmic_bytes(cls, N, C, fp32)
        t = traffic.get(cls)
        hbm[cls] = {"avg_ms": ms, "achieved_GBps": b / (ms * 1e-3) / 1e9,
                    "frac": b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                    "traffic_bytes": t,
                    "traffic_GBps": (t / (ms * 1e-3) / 1e9) if t else None}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        import oracle
        box_o = oracle.Box(L=W["L"], m0=W["m0"], eps0=W["eps0"])
        cpu = cpu_baseline(W, ics, box_o)

    mf = force_rate(ctx, box, st, W, dz, torch) if not args.no_force_rate else None
    ms_per_step = 1e3 * t_main / K
    out = {
        "metric": METRIC, "value": N * K / t_main, "unit": UNIT, "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": (f"{W['n_side']}^3 particles, L={W['L']:g} Mpc/h, mesh "
                                f"{W['ng']}^3, Zel'dovich z=49 BBKS seed {W['seed']}, "
                                f"{K} of {W['n_steps']} log KDK steps to z=0, DZS 2x2x2 "
                                f"(l_max {W['lmax_over_lambda']} lambda) + lightcone, "
                                f"tree theta {W['theta_tree']}, "
                                + ("precision form (FP32 pair/mesh/FFT, FP64 state)" if fp32
                                   else "FP64 plain form")
                                + (f", individual power-of-two steps (2^{args.hier} sub-steps, "
                                   f"eta {args.eta}, out-of-lightcone limiter"
                                   + (", PM on the global step only" if args.pm_global else "")
                                   + ")" if args.hier else "")),
                   "preset": args.workload, "particles": N, "mesh": W["ng"], "box": W["L"],
                   "parallelism": "1 GPU"},
        "roofline": roofline, "hbm_kernels": hbm, "cpu_baseline": cpu, "twin": twin,
        "force_rate": mf,
        "pair_interactions_per_step": pairs / K, "lightcone_records": n_records,
        "particles_final": n_final,
        "kernels_ms_per_step": {c: round(v / K, 4) for c, v in sorted(totals.items(),
                                                                    key=lambda kv: -kv[1])},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

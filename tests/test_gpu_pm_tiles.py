"""The LDS tiles of the PM deposit and interpolation against the direct kernels (paper Sec.
2.1: cloud-in-cell assignment and interpolation of the mesh force).

Deposit: both paths add the same 32.32 fixed-point contributions with integer atomics, so the
mesh is the same integer sum.  Interpolation: both paths evaluate the same 4-point differences
and weights in the same order, from the same potential values (read from LDS or from the
mesh).  So every force must be bit-identical for every tile_chunk: no tiles (-1), each chunk
size, and the default (0).  The PM force of the tiled path is also checked against the FP64
oracle at the PM bar (1e-8).  Inputs are put in key order first, as the step does before its
force, so that chunks are compact and the tiles are used; a host mirror of the kernels' fit
rules asserts that both the tiles and the direct fallback are exercised.
"""
import math
import sys

import numpy as np
import pytest

import dzs_ics
import oracle

pytestmark = pytest.mark.gpu

L, NG = 100.0, 64
TILE = 4096
CHUNKS = [256, 1024, 4096, 16384]


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
    c = dz.Context(max_particles=70000, max_mesh_side=NG)
    yield c
    c.close()


def _case(kind):
    if kind == "clustered":
        return dzs_ics.clustered_random(60000, L, seed=71, r_clump=L / 80)
    if kind == "zeldovich":
        return dzs_ics.zeldovich(32, L, 0.02, seed=72, spectrum="powerlaw")
    # a clump around the box corner (its clouds wrap on every axis) plus particles on the last
    # representable coordinate below L, whose base index may round to N_g
    ps = dzs_ics.clustered_random(40000, L, seed=73, r_clump=L / 40, n_clumps=1, frac=1.0)
    c = np.array([ps.x.mean(), ps.y.mean(), ps.z.mean()])
    for a, k in enumerate(("x", "y", "z")):
        setattr(ps, k, np.mod(getattr(ps, k) - c[a], L))
    edge = np.nextafter(L, 0.0)
    ps.x[:50] = edge
    ps.y[25:75] = edge
    ps.z[::997] = edge
    ps.mult[::13] = 37
    return ps


def _fits(x, y, z, n, chunk, pad, ng):
    """Which chunks a kernel tiles in LDS: the unwrapped base indices floor(x / Delta) of a
    chunk, widened by `pad` points per axis (deposit: base + 1, pad 2; interpolation: base - 2
    .. base + 3, pad 6), span at most TILE points.  The interpolation uses tiles only when the
    particles are at least half as many as the mesh points."""
    if pad == 6 and 2 * n < ng ** 3:
        return np.zeros(0, bool)
    delta = L / ng
    out = []
    for p0 in range(0, n, chunk):
        sl = slice(p0, min(n, p0 + chunk))
        ext = [int(np.floor(v[sl] / delta).max() - np.floor(v[sl] / delta).min()) + pad
               for v in (x, y, z)]
        out.append(ext[0] * ext[1] * ext[2] <= TILE)
    return np.array(out)


@pytest.mark.parametrize("kind,ng", [("clustered", 64), ("clustered", 32), ("zeldovich", 64),
                                     ("zeldovich", 32), ("corner", 64), ("corner", 32)])
def test_tile_chunks_give_identical_forces(dz, ctx, kind, ng):
    import torch
    r_s = 1.25 * L / ng
    ps = _case(kind)
    n = ps.n
    m0 = dzs_ics.particle_mass(L, 32 ** 3)
    box = dz.make_box(L, m0, L / 32 / 40)
    obox = oracle.Box(L=L, m0=m0, eps0=L / 32 / 40)
    st = dz.State.from_host(ps)
    ctx.sort_state(box, st, ties_by_id=True)
    torch.cuda.synchronize()
    h = st.to_host()
    _log(f"PM tiles kind={kind} n={n} mesh {ng}")

    def force(chunk):
        ctx.pm_force(box, st, dz.PMParams(ng, dz.DZS_FP64, r_s, 0, chunk))
        torch.cuda.synchronize()
        return np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(),
                         st.gz[:n].cpu().numpy()])

    g_direct = force(-1)
    n_fit = {2: 0, 6: 0}
    for chunk in CHUNKS + [0]:
        g = force(chunk)
        assert np.array_equal(g, g_direct), chunk
        if chunk:
            for pad in (2, 6):
                fit = _fits(h["x"], h["y"], h["z"], n, chunk, pad, ng)
                n_fit[pad] += int(fit.sum())
                _log(f"  chunk {chunk}, pad {pad}: {int(fit.sum())} of {fit.size} chunks in LDS")
    # on the 64^3 mesh (more points than twice the particles) the interpolation reads the
    # mesh directly; on the 32^3 mesh it uses tiles
    assert n_fit[2] > 0 and (n_fit[6] > 0 or ng == 64)
    ref = oracle.pm_force(h["x"], h["y"], h["z"], h["mult"], obox, ng, r_s)
    err = math.sqrt(np.mean(np.sum((g_direct - ref) ** 2, 0)) / np.mean(np.sum(ref ** 2, 0)))
    _log(f"  pm rms rel err {err:.3e}")
    assert err <= 1e-8


def test_tiles_of_an_unsorted_state_match(dz, ctx):
    """Out of key order the chunks are scattered and mostly add directly: same forces."""
    import torch
    ps = _case("clustered")
    n = ps.n
    box = dz.make_box(L, dzs_ics.particle_mass(L, 32 ** 3), L / 32 / 40)
    st = dz.State.from_host(ps)
    out = []
    for chunk in (-1, 256, 0):
        ctx.pm_force(box, st, dz.PMParams(32, dz.DZS_FP64, 1.25 * L / 32, 0, chunk))
        torch.cuda.synchronize()
        out.append(np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(),
                             st.gz[:n].cpu().numpy()]))
    fit = _fits(ps.x, ps.y, ps.z, n, 256, 2, 32)
    _log(f"unsorted: {int(fit.sum())} of {fit.size} chunks of 256 binned in LDS")
    assert np.array_equal(out[1], out[0]) and np.array_equal(out[2], out[0])


def test_tile_chunk_fp32_mesh(dz, ctx):
    """The precision form (FP32 potential in the tiles): identical forces too."""
    import torch
    ps = _case("clustered")
    n = ps.n
    box = dz.make_box(L, dzs_ics.particle_mass(L, 32 ** 3), L / 32 / 40)
    st = dz.State.from_host(ps)
    ctx.sort_state(box, st)
    out = []
    for chunk in (-1, 256, 1024):
        ctx.pm_force(box, st, dz.PMParams(32, dz.DZS_FP32, 1.25 * L / 32, 0, chunk))
        torch.cuda.synchronize()
        out.append(np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(),
                             st.gz[:n].cpu().numpy()]))
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_tile_chunk_rejects(dz, ctx):
    ps = _case("zeldovich")
    box = dz.make_box(L, dzs_ics.particle_mass(L, ps.n), L / 32 / 40)
    st = dz.State.from_host(ps)
    for bad in (-2, 1, 128, 300, 768, 32768):
        with pytest.raises(dz.DZSError):
            ctx.pm_force(box, st, dz.PMParams(NG, dz.DZS_FP64, 1.25 * L / NG, 0, bad))

"""The LDS-binned cloud-in-cell deposit against the direct one (paper Sec. 2.1, the PM density
assignment).

Both paths add the same 32.32 fixed-point contributions with integer atomics, so the mesh, and
every force computed from it, must be bit-identical for every deposit_chunk: the direct
deposit (-1), the tiled one at each chunk size, and the default (0).  The PM force of the
tiled path is also checked against the FP64 oracle at the PM bar (1e-8).  Inputs are put in
key order first, as the step does before its force, so that chunks are compact and the tile
path runs; a host mirror of the kernel's fit rule asserts that both the tile path and the
fallback are exercised.
"""
import math
import sys

import numpy as np
import pytest

import dzs_ics
import oracle

pytestmark = pytest.mark.gpu

L, NG = 100.0, 64
R_S = 1.25 * L / NG
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


def _fits(x, y, z, n, chunk):
    """Which chunks the kernel bins in LDS: the unwrapped base indices floor(x / Delta) of a
    chunk span at most TILE points, counting base + 1 on every axis."""
    delta = L / NG
    out = []
    for p0 in range(0, n, chunk):
        sl = slice(p0, min(n, p0 + chunk))
        ext = [int(np.floor(v[sl] / delta).max() - np.floor(v[sl] / delta).min()) + 2
               for v in (x, y, z)]
        out.append(ext[0] * ext[1] * ext[2] <= TILE)
    return np.array(out)


@pytest.mark.parametrize("kind", ["clustered", "zeldovich", "corner"])
def test_deposit_chunks_give_identical_forces(dz, ctx, kind):
    import torch
    ps = _case(kind)
    n = ps.n
    m0 = dzs_ics.particle_mass(L, 32 ** 3)
    box = dz.make_box(L, m0, L / 32 / 40)
    obox = oracle.Box(L=L, m0=m0, eps0=L / 32 / 40)
    st = dz.State.from_host(ps)
    ctx.sort_state(box, st, ties_by_id=True)
    torch.cuda.synchronize()
    h = st.to_host()
    _log(f"deposit kind={kind} n={n}")

    def force(chunk):
        ctx.pm_force(box, st, dz.PMParams(NG, dz.DZS_FP64, R_S, 0, chunk))
        torch.cuda.synchronize()
        return np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(),
                         st.gz[:n].cpu().numpy()])

    g_direct = force(-1)
    n_fit = 0
    for chunk in CHUNKS + [0]:
        g = force(chunk)
        assert np.array_equal(g, g_direct), chunk
        if chunk:
            fit = _fits(h["x"], h["y"], h["z"], n, chunk)
            n_fit += int(fit.sum())
            _log(f"  chunk {chunk}: {int(fit.sum())} of {fit.size} chunks binned in LDS")
    assert n_fit > 0
    ref = oracle.pm_force(h["x"], h["y"], h["z"], h["mult"], obox, NG, R_S)
    err = math.sqrt(np.mean(np.sum((g_direct - ref) ** 2, 0)) / np.mean(np.sum(ref ** 2, 0)))
    _log(f"  pm rms rel err {err:.3e}")
    assert err <= 1e-8


def test_deposit_of_an_unsorted_state_matches(dz, ctx):
    """Out of key order the chunks are scattered and mostly add directly: same forces."""
    import torch
    ps = _case("clustered")
    n = ps.n
    box = dz.make_box(L, dzs_ics.particle_mass(L, 32 ** 3), L / 32 / 40)
    st = dz.State.from_host(ps)
    out = []
    for chunk in (-1, 256, 0):
        ctx.pm_force(box, st, dz.PMParams(NG, dz.DZS_FP64, R_S, 0, chunk))
        torch.cuda.synchronize()
        out.append(np.stack([st.gx[:n].cpu().numpy(), st.gy[:n].cpu().numpy(),
                             st.gz[:n].cpu().numpy()]))
    fit = _fits(ps.x, ps.y, ps.z, n, 256)
    _log(f"unsorted: {int(fit.sum())} of {fit.size} chunks of 256 binned in LDS")
    assert np.array_equal(out[1], out[0]) and np.array_equal(out[2], out[0])


def test_deposit_chunk_fp32_mesh(dz, ctx):
    """The precision form reads the same fixed-point mesh: identical forces too."""
    import torch
    ps = _case("clustered")
    n = ps.n
    box = dz.make_box(L, dzs_ics.particle_mass(L, 32 ** 3), L / 32 / 40)
    st = dz.State.from_host(ps)
    ctx.sort_state(box, st)
    out = []
    for chunk in (-1, 1024):
        ctx.pm_force(box, st, dz.PMParams(NG, dz.DZS_FP32, R_S, 0, chunk))
        torch.cuda.synchronize()
        out.append(st.gx[:n].cpu().numpy().copy())
    assert np.array_equal(out[0], out[1])


def test_deposit_chunk_rejects(dz, ctx):
    ps = _case("zeldovich")
    box = dz.make_box(L, dzs_ics.particle_mass(L, ps.n), L / 32 / 40)
    st = dz.State.from_host(ps)
    for bad in (-2, 1, 128, 300, 768, 32768):
        with pytest.raises(dz.DZSError):
            ctx.pm_force(box, st, dz.PMParams(NG, dz.DZS_FP64, R_S, 0, bad))

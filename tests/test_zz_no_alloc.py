"""The allocation-free PM entry point (pm_force_noalloc) against pm_force through a context:
the same kernels on the same inputs, so the same bits, on two calls in a row (the second with
fewer particles and a smaller mesh), in both forms; a mesh side beyond the static array's
capacity is refused."""
import sys

import numpy as np
import pytest

import dzs_ics

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("fp32", [False, True])
def test_pm_force_noalloc_matches_pm_force(fp32):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2005_05328_amd as dz
    prec = dz.DZS_FP32 if fp32 else dz.DZS_FP64
    L = 100.0
    cases = [(20000, 64, 21), (3000, 32, 22)]   # the second call smaller
    ctx = dz.Context(20000, 64)
    for n, ng, seed in cases:
        ps = dzs_ics.merged_state(dzs_ics.clustered_random(n, L, seed=seed, r_clump=L / 50),
                                  seed=seed + 1, max_mult=16)
        box = dz.make_box(L, dzs_ics.particle_mass(L, n), L / 27 / 40)
        prm = dz.PMParams(ng, prec, 1.25 * L / ng, 0, 0)
        a = dz.State.from_host(ps)
        b = dz.State.from_host(ps)
        ctx.pm_force(box, a, prm)
        dz.pm_force_noalloc(box, b, prm)
        torch.cuda.synchronize()
        for k in ("gx", "gy", "gz"):
            ga, gb = getattr(a, k)[:n].cpu().numpy(), getattr(b, k)[:n].cpu().numpy()
            assert np.array_equal(ga, gb), (n, ng, k)
            assert np.abs(ga).max() > 0.0
        # accumulate adds onto what g holds
        prm.accumulate = 1
        dz.pm_force_noalloc(box, b, prm)
        torch.cuda.synchronize()
        assert np.array_equal(b.gx[:n].cpu().numpy(), 2.0 * a.gx[:n].cpu().numpy())
        _log(f"noalloc PM n={n} ng={ng} fp32={fp32}: identical to pm_force")
    ctx.close()
    big = dz.PMParams(96, prec, 1.25 * L / 96, 0, 0)
    with pytest.raises(dz.DZSError):
        dz.pm_force_noalloc(box, b, big)

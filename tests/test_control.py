"""Host logic of the library (no GPU needed): the run-halt conditions (paper Sec. 4.1.1) and
the speed-up forecast of Sec. 4.2 (eqs. 6-7).

The forecast is pinned against the oracle's independent comoving distance (scipy quadrature):
a_DZS must put half the box volume inside the lightcone sphere; r must take its two anchor
values at the two reference runs' particle masses and stay at 0.4 for coarser ones.
"""
import math

import pytest

import oracle

dz = pytest.importorskip("paper_2005_05328_amd")

M_LARGE = 0.3 * 27.75366 * 8192.0 ** 3 / 512 ** 3
M_SMALL = 0.3 * 27.75366 * 512.0 ** 3 / 512 ** 3


@pytest.mark.parametrize("L,N", [(4000.0, 4e12), (8192.0, 512 ** 3), (512.0, 512 ** 3),
                                 (2000.0, 2048 ** 3), (128.0, 512 ** 3)])
def test_forecast_half_volume_and_power(L, N):
    f = dz.forecast_speedup(L, N)
    # 4/3 pi chi(a_DZS)^3 = L^3 / 2 with the oracle's chi
    assert abs(4.0 / 3.0 * math.pi * oracle.chi(f.a_dzs) ** 3 / L ** 3 - 0.5) < 1e-9
    m = 0.3 * 27.75366 * L ** 3 / N
    assert abs(f.particle_mass / m - 1.0) < 1e-12
    r = max(0.4, 0.4 + 0.6 * (m - M_LARGE) / (M_SMALL - M_LARGE))
    assert abs(f.r - r) < 1e-12
    assert f.speedup == pytest.approx(f.a_dzs ** -f.r, rel=1e-14)


def test_forecast_anchors_and_trends():
    assert dz.forecast_speedup(8192.0, 512 ** 3).r == pytest.approx(0.4, abs=1e-12)
    assert dz.forecast_speedup(512.0, 512 ** 3).r == pytest.approx(1.0, abs=1e-12)
    # coarser than the coarsest reference run: held at 0.4
    assert dz.forecast_speedup(16384.0, 256 ** 3).r == 0.4
    # at a fixed particle mass the gain grows with the box (earlier a_DZS)
    gains = [dz.forecast_speedup(L, (L / 2.0) ** 3).speedup for L in (500.0, 1000.0, 2000.0,
                                                                       4000.0, 8000.0)]
    assert all(b > a for a, b in zip(gains, gains[1:]))
    # a sphere holding half the box before a = 1e-4 is rejected
    with pytest.raises(dz.DZSError):
        dz.forecast_speedup(1e5, 1e9)


def test_halt_conditions():
    H = dz
    base = dict(max_balance=1.1, min_ratio=0.3, runtime_limit_s=3600.0, restart_window_s=1800.0)
    # nothing holds
    assert dz.halt_check(1.05, 0.6, 0.61, 1000.0, 900.0, **base) == 0
    # workload balance above its threshold
    assert dz.halt_check(1.2, 0.6, 0.61, 1000.0, 900.0, **base) == H._abi.DZS_HALT_BALANCE
    # R below its threshold
    assert dz.halt_check(1.0, 0.29, 0.31, 1000.0, 900.0, **base) == H._abi.DZS_HALT_RATIO
    # at the run-time limit, R falling 0.1 per 1000 s from 0.45: 0.45 - 0.18 = 0.27 < 0.3
    # within the 1800 s window -> halt now; a slower fall (0.01 per 1000 s) does not
    assert dz.halt_check(1.0, 0.45, 0.55, 3600.0, 2600.0, **base) == H._abi.DZS_HALT_PREDICTED
    assert dz.halt_check(1.0, 0.45, 0.46, 3600.0, 2600.0, **base) == 0
    # the same fall before the limit is not a reason
    assert dz.halt_check(1.0, 0.45, 0.55, 3000.0, 2000.0, **base) == 0
    # balance condition off (<= 0), run-time limit off
    assert dz.halt_check(5.0, 0.9, 0.9, 1e9, 0.0, 0.0, 0.3, 0.0, 100.0) == 0
    # several reasons at once
    both = dz.halt_check(1.5, 0.2, 0.25, 4000.0, 3000.0, **base)
    assert both == (H._abi.DZS_HALT_BALANCE | H._abi.DZS_HALT_RATIO | H._abi.DZS_HALT_PREDICTED)


def test_ensemble_repack_and_control_on_host_tensors():
    """The re-pack keeps each box's survivors, in order, in consecutive ranges of a state
    fitted to their total; the control reports the ratio to the last packing and asks for a
    re-pack once it falls under the threshold (CPU tensors: the re-pack is plain copies)."""
    import torch
    from paper_2005_05328_amd import ensemble
    first, counts = [0, 5, 5, 12], [3, 0, 4]
    st = dz.State(12, device="cpu")
    for k in ensemble._ARR:
        t = getattr(st, k)
        t.copy_(torch.arange(12).to(t.dtype) + (100 if k == "id" else 0))
    st.n = 12
    out, nf = ensemble.repack(st, first, counts, device="cpu")
    assert nf == [0, 3, 3, 7] and out.n == out.capacity == 7
    assert out.id.tolist() == [100, 101, 102, 105, 106, 107, 108]
    assert out.x.tolist() == [0.0, 1.0, 2.0, 5.0, 6.0, 7.0, 8.0]
    out2, _ = ensemble.repack(st, first, counts, capacity=20, device="cpu")
    assert out2.capacity == 20 and out2.n == 7
    r, why = ensemble.control(counts, 12, min_ratio=0.9)
    assert r == pytest.approx(7 / 12) and why == dz._abi.DZS_HALT_RATIO
    r, why = ensemble.control([5, 0, 6], 12, min_ratio=0.9)
    assert why == 0

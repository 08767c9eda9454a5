"""Host-side checks of the C ABI (no GPU needed).

* libdzs.so loads and exports every function include/dzs.h declares;
* the ctypes mirror has the sizes of the C structs' fields as declared;
* dzs_step_factors (host quadrature + Chebyshev series) agrees with the oracle's cosmology
  within 1e-13 and its Chebyshev series reproduce chi(a) and D(a0, a) inside the step;
* argument errors are reported as status codes, not crashes.
"""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "dzs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", txt,
                                 flags=re.M)))


def test_library_exports_every_declared_symbol():
    import paper_2005_05328_amd as dz
    declared = _declared_functions()
    assert {"dzs_coarsen", "pm_force", "tree_force", "kdk_step", "lightcone_emit"} <= set(declared)
    L = dz.lib()
    for name in declared:
        assert hasattr(L, name), name
    from paper_2005_05328_amd import _abi
    assert set(_abi.EXPORTS) == set(declared)


def test_record_and_struct_layout():
    from paper_2005_05328_amd import _abi
    assert C.sizeof(_abi.LCRecord) == 64
    assert C.sizeof(_abi.Box) == 32
    assert C.sizeof(_abi.Particles) == 12 * 8 + 16
    assert C.sizeof(_abi.LCParams) == 3 * 8 + 5 * 8 + 8 + 2 * 24 * 8
    assert C.sizeof(_abi.Capacity) == 8 + 4 * 4
    assert C.sizeof(_abi.TreeParams) == 3 * 8 + 6 * 4 + 8
    assert C.sizeof(_abi.HierParams) == 2 * 4 + 5 * 8 + 2 * 4


@pytest.mark.parametrize("a0,a1", [(0.02, 0.02 * math.exp(0.07824)), (0.5, 0.55),
                                   (0.9247, 1.0), (0.7908, 0.8551)])
def test_step_factors_match_oracle_cosmology(a0, a1):
    import paper_2005_05328_amd as dz
    sp = dz.step_factors(a0, a1, 0.3)
    ref = oracle.step_factors(a0, a1)
    assert abs(sp.K1 - ref["K1"]) <= 1e-13 * ref["K1"]
    assert abs(sp.K2 - ref["K2"]) <= 1e-13 * ref["K2"]
    assert abs(sp.lc.D - ref["D"]) <= 1e-13 * ref["D"]
    assert abs(sp.lc.chi2_0 - ref["chi2_0"]) <= 2e-13 * ref["chi2_0"]
    assert abs(sp.lc.chi2_1 - ref["chi2_1"]) <= 2e-13 * max(ref["chi2_1"], 1.0)
    # Chebyshev series inside the step
    n = sp.lc.n_cheb
    cc = np.array(sp.lc.cheb_chi[:n])
    cd = np.array(sp.lc.cheb_drift[:n])
    for t in np.linspace(-1, 1, 9):
        a = a0 + 0.5 * (t + 1) * (a1 - a0)
        chi_ref = oracle.chi(a) if a < 1 else 0.0
        d_ref = oracle.drift_factor(a0, a) if a > a0 else 0.0
        chi_c = np.polynomial.chebyshev.chebval(t, cc)
        d_c = np.polynomial.chebyshev.chebval(t, cd)
        assert abs(chi_c - chi_ref) <= 1e-12 * max(chi_ref, 1.0)
        assert abs(d_c - d_ref) <= 1e-13 * ref["D"]


def test_step_factors_rejects_bad_input():
    import paper_2005_05328_amd as dz
    with pytest.raises(dz.DZSError):
        dz.step_factors(0.5, 0.4)
    with pytest.raises(dz.DZSError):
        dz.step_factors(0.5, 1.2)


def test_null_context_is_an_error_not_a_crash():
    import paper_2005_05328_amd as dz
    L = dz.lib()
    box = dz.Box(100.0, 1.0, 0.1, 43.0091)
    from paper_2005_05328_amd import _abi
    p = _abi.Particles()
    assert L.pm_force(None, C.byref(box), C.byref(p), None, None) == _abi.DZS_EINVAL
    assert L.tree_force(None, C.byref(box), C.byref(p), None, None, 0, None) == _abi.DZS_EINVAL
    assert L.dzs_ctx_destroy(None) == _abi.DZS_EINVAL
    h = C.c_void_p()
    assert L.dzs_ctx_create(C.byref(h), 0, None) == _abi.DZS_EINVAL


def test_header_constants_match_the_binding():
    """Every #define of include/dzs.h that the ctypes mirror repeats has the same value."""
    from paper_2005_05328_amd import _abi
    txt = open(os.path.join(ROOT, "include", "dzs.h")).read()
    defs = dict(re.findall(r"^#define\s+(DZS_[A-Z0-9_]+)\s+\(?(-?\d+)u?\)?", txt, flags=re.M))
    shared = [k for k in defs if hasattr(_abi, k)]
    assert {"DZS_PM_CHUNK_MIN", "DZS_PM_CHUNK_MAX", "DZS_PM_CHUNK_DEFAULT",
            "DZS_FP32", "DZS_BATCH_MAX"} <= set(shared)
    for k in shared:
        assert getattr(_abi, k) == int(defs[k]), k


def test_library_matches_its_sources_and_a_stale_one_is_refused(monkeypatch):
    from paper_2005_05328_amd import _abi
    L = _abi.load()
    assert L.dzs_source_hash().decode() == _abi._source_hash()
    monkeypatch.setattr(_abi, "_source_hash", lambda: "0" * 16)
    with pytest.raises(ImportError, match="other sources"):
        _abi.load()

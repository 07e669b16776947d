"""CPU checks of the C-ABI library: it loads, exports every symbol declared in
include/amber.h, and its host-side history logic agrees with the oracle (no GPU
work is done here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _amber():
    import paper_2109_10375_amd as amber
    if not os.path.exists(amber.library_path()):
        from paper_2109_10375_amd import build
        build.build()
    return amber


def _declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "amber.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**(amber_[a-z_0-9]+)\(", hdr, re.M)))


def test_header_declares_the_stages():
    syms = _declared_symbols()
    for s in ("amber_radiation", "amber_zre", "amber_rank", "amber_plan_create", "amber_workspace_bytes",
              "amber_status", "amber_weibull_fit", "amber_weibull_table"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    amber = _amber()
    L = amber.lib()
    for s in _declared_symbols():
        assert hasattr(L, s), s
    assert set(_declared_symbols()) <= set(amber._lib.SYMBOLS) | {"amber_version"}
    assert b"gfx950" in L.amber_version()


def test_no_torch_types_in_header():
    hdr = open(os.path.join(ROOT, "include", "amber.h")).read()
    assert "torch" not in hdr.lower().replace("pytorch", "")
    assert "at::" not in hdr and "Tensor" not in hdr


def test_strerror_codes():
    L = _amber().lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.amber_strerror(code)


@pytest.mark.parametrize("hist", [(8.0, 4.0, 3.0), (7.95, 4.68, 2.90), (7.91, 5.45, 2.69),
                                  (7.83, 6.54, 2.33), (6.0, 2.0, 1.5), (10.0, 6.0, 4.0), (9.0, 3.0, 1.0)])
def test_library_weibull_fit_matches_oracle(hist):
    """Appendix A solved independently on both sides (secant vs Brent)."""
    amber = _amber()
    w = amber.History.fit_host(*hist)
    a, b, c = oracle.weibull_fit(*hist)
    assert abs(w.a_w - a) <= 1e-12 * a and abs(w.b_w - b) <= 1e-12 * b and abs(w.c_w - c) <= 1e-12 * c


@pytest.mark.parametrize("bad", [(8.0, 4.0, 0.5), (8.0, 4.0, 16.0), (8.0, 0.0, 3.0), (1.0, 6.0, 3.0)])
def test_library_weibull_rejects(bad):
    amber = _amber()
    with pytest.raises(amber.AmberError):
        amber.History.fit_host(*bad)


def test_table_geometry_and_values_identical_to_oracle():
    """Given the same coefficients, the library's table (host code) and the
    oracle's table are the same bytes; so are h, T and z_top."""
    amber = _amber()
    L = amber.lib()
    for hist in [(8.0, 4.0, 3.0), (7.83, 6.54, 2.33), (10.0, 6.0, 4.0)]:
        H = oracle.History.from_params(*hist)
        w = amber._lib.AmberWeibull()
        assert L.amber_weibull_from_coeffs(H.a, H.b, H.c, ctypes.byref(w)) == 0
        assert w.h == H.h and w.z_top == H.z_top and w.table_n == H.T + 1
        tab = np.empty(w.table_n, dtype=np.float64)
        assert L.amber_weibull_table(ctypes.byref(w), tab.ctypes.data_as(ctypes.c_void_p), w.table_n) == 0
        assert np.array_equal(tab, H.X)


def test_plan_rejects_unsupported_sizes_without_gpu():
    amber = _amber()
    L = amber.lib()
    h = ctypes.c_void_p()
    for n in (0, 7, 100, 2048):
        assert L.amber_plan_create(ctypes.byref(h), n, 100.0) == amber._lib.E_SIZE


def test_package_has_no_cpu_fallback():
    """The binding raises when the library is absent instead of computing."""
    src = open(os.path.join(ROOT, "paper_2109_10375_amd", "_lib.py")).read()
    assert "import oracle" not in src and "numpy" not in src
    assert "no CPU fallback" in src


def test_batch_entry_points_check_their_arguments_on_the_host():
    amber = _amber()
    L = amber.lib()
    assert "amber_batch_run" in _declared_symbols() and "amber_batch_workspace_bytes" in _declared_symbols()
    Item = amber._lib.AmberBatchItem
    assert L.amber_batch_workspace_bytes(None, 0) == 0
    items = (Item * 1)()
    assert L.amber_batch_workspace_bytes(items, 1) == 0  # no plan
    assert L.amber_batch_run(None, 1, None, None, 0, None) == amber._lib.E_ARG
    assert L.amber_batch_run(items, 0, None, ctypes.c_void_p(1), 1, None) == amber._lib.E_ARG
    # an item with no plan is rejected before anything is enqueued
    assert L.amber_batch_run(items, 1, None, ctypes.c_void_p(1), 1, None) == amber._lib.E_ARG


@pytest.mark.parametrize("hist,z_mid", [((8.0, 4.0, 3.0), 8.0), ((7.83, 6.54, 2.33), 7.83), ((9.0, 2.0, 1.5), 9.0)])
def test_growth_table_identical_to_oracle(hist, z_mid):
    """The library's growth ratios at the table nodes equal the oracle's byte
    for byte (the same series, written separately on each side), so growth
    matching can be compared bit for bit."""
    amber = _amber()
    H = oracle.History.from_params(*hist)
    w = amber._lib.AmberWeibull()
    assert amber.lib().amber_weibull_from_coeffs(H.a, H.b, H.c, ctypes.byref(w)) == 0
    g_lib = amber.History.growth_table_host(w, z_mid).numpy()
    g_or = oracle.growth_table(H, z_mid)
    assert g_lib.shape == g_or.shape
    assert np.array_equal(g_lib.view(np.uint64), g_or.view(np.uint64))


def test_serving_busy_time_is_the_union_of_batch_intervals():
    from paper_2109_10375_amd.serve import _union
    assert _union([]) == 0.0
    assert _union([(0.0, 1.0), (0.5, 2.0), (3.0, 4.0)]) == pytest.approx(3.0)
    assert _union([(1.0, 2.0), (0.0, 5.0)]) == pytest.approx(5.0)

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
              "amber_status", "amber_weibull_fit", "amber_weibull_table", "amber_history_prepare",
              "amber_batch_run", "amber_strerror", "amber_plan_destroy"):
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
    assert L.amber_batch_workspace_bytes(None, 0, 1) == 0
    items = (Item * 1)()
    assert L.amber_batch_workspace_bytes(items, 1, 1) == 0  # no plan
    assert L.amber_batch_workspace_bytes(items, 1, 17) == 0  # too many lanes
    assert L.amber_batch_run(None, 1, None, None, 0, None, None) == amber._lib.E_ARG
    assert L.amber_batch_run(items, 0, None, ctypes.c_void_p(1), 1, None, None) == amber._lib.E_ARG
    # an item with no plan is rejected before anything is enqueued
    assert L.amber_batch_run(items, 1, None, ctypes.c_void_p(1), 1, None, None) == amber._lib.E_ARG
    ex = ctypes.c_void_p()
    assert L.amber_executor_create(ctypes.byref(ex), 0) == amber._lib.E_ARG
    assert L.amber_executor_create(ctypes.byref(ex), 17) == amber._lib.E_ARG


@pytest.mark.parametrize("hist,z_mid,om", [((8.0, 4.0, 3.0), 8.0, 0.3), ((7.83, 6.54, 2.33), 7.83, 0.3),
                                           ((9.0, 2.0, 1.5), 9.0, 0.3), ((8.0, 4.0, 3.0), 8.0, 0.1),
                                           ((8.0, 4.0, 3.0), 8.0, 1.0)])
def test_growth_table_matches_oracle_quadrature(hist, z_mid, om):
    """The library's growth ratios G_j = D(z_j)/D(z_mid) (its own
    hypergeometric series) agree with the oracle's Gauss-Legendre quadrature
    of the growing-mode integral to 1e-12 relative at every node, and the
    pairs' X_j are the library's inversion table bit for bit."""
    amber = _amber()
    H = oracle.History.from_params(*hist)
    w = amber._lib.AmberWeibull()
    assert amber.lib().amber_weibull_from_coeffs(H.a, H.b, H.c, ctypes.byref(w)) == 0
    pairs = amber.History.growth_table_host(w, z_mid, om).numpy()
    g_lib, x_lib = pairs[1::2], pairs[0::2]
    g_or = oracle.growth_table(H, z_mid, om)
    assert g_lib.shape == g_or.shape
    rel = np.max(np.abs(g_lib / g_or - 1.0))
    print(f"growth table vs oracle quadrature: max relative difference {rel:.2e}")
    assert rel <= 1e-12
    x_tab = np.empty(w.table_n, dtype=np.float64)
    assert amber.lib().amber_weibull_table(ctypes.byref(w), x_tab.ctypes.data_as(ctypes.c_void_p), w.table_n) == 0
    assert np.array_equal(x_lib.view(np.uint64), x_tab.view(np.uint64))


def test_serving_busy_time_is_the_union_of_batch_intervals():
    from paper_2109_10375_amd.serve import _union
    assert _union([]) == 0.0
    assert _union([(0.0, 1.0), (0.5, 2.0), (3.0, 4.0)]) == pytest.approx(3.0)
    assert _union([(1.0, 2.0), (0.0, 5.0)]) == pytest.approx(5.0)


# In-register DFT sizes the FFT passes support (products of 2, 3 and 4 up to 32).
_DFT_SIZES = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32}


@pytest.mark.parametrize("n", [8, 16, 32, 64, 96, 128, 192, 256, 512, 1024])
def test_fft_schedule_candidates_are_valid_splits(n):
    """Every compiled candidate splits its transform as L1 x L2 with L1 | L2,
    both among the in-register DFT sizes, tiles that cover the spectrum rows
    exactly and blocks within 1024 threads (host-only queries)."""
    import paper_2109_10375_amd as amber
    cand = amber.fft_schedules(n)
    assert len(cand["col"]) >= 1 and len(cand["z"]) >= 1
    assert len(set(cand["col"])) == len(cand["col"]) and len(set(cand["z"])) == len(cand["z"])
    for n1, c in cand["col"]:
        n2 = n // n1
        assert n1 * n2 == n and n2 % n1 == 0 and n1 in _DFT_SIZES and n2 in _DFT_SIZES
        assert (n // 2) % c == 0 and n1 * c <= 1024
    for m1, zl in cand["z"]:
        m = n // 2
        m2 = m // m1
        assert m1 * m2 == m and m2 % m1 == 0 and m1 in _DFT_SIZES and m2 in _DFT_SIZES
        assert m1 * zl <= 1024
    a, b = ctypes.c_int(), ctypes.c_int()
    L = amber.lib()
    assert L.amber_fft_schedule_info(n, 0, len(cand["col"]), ctypes.byref(a), ctypes.byref(b)) == -1
    assert L.amber_fft_schedule_info(n, 1, len(cand["z"]), ctypes.byref(a), ctypes.byref(b)) == -1
    assert L.amber_fft_schedule_info(n, 2, 0, ctypes.byref(a), ctypes.byref(b)) == -1
    assert L.amber_fft_schedule_info(n, 0, -1, ctypes.byref(a), ctypes.byref(b)) == -1
    assert L.amber_fft_schedules(n + 1, ctypes.byref(a), ctypes.byref(b)) == -2


def test_tune_cache_round_trip_and_stale_entries(tmp_path):
    from paper_2109_10375_amd import tune
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load(path) == {}
    cand = {"col": [(32, 8), (32, 4)], "z": [(16, 16), (16, 8)]}
    key = tune.entry_key("gfx950|cu256|288GiB", 1024)
    entry = {"col": 1, "z": 0, "col_split": [32, 4], "z_split": [16, 16], "ms": [[1.0, 2.0], [0.5, 3.0]], "reps": 5}
    tune.store(path, key, entry)
    tune.store(path, tune.entry_key("gfx950|cu256|288GiB", 512), dict(entry, col=0, col_split=[32, 8]))
    got = tune.load(path)
    assert got[key] == entry and len(got) == 2
    assert tune.valid_entry(got[key], cand)
    assert not tune.valid_entry(dict(entry, col=2), cand)                 # no such candidate
    assert not tune.valid_entry(dict(entry, col_split=[32, 16]), cand)    # candidate list changed
    assert not tune.valid_entry({"col": 0}, cand)
    with open(path, "w") as f:
        f.write("{not json")
    assert tune.load(path) == {}
    with open(path, "w") as f:
        f.write('{"version": 0, "entries": {}}')
    assert tune.load(path) == {}


def _kernel_poly_from_source():
    src = open(os.path.join(ROOT, "paper_2109_10375_amd", "csrc", "fft.hip")).read()
    body = re.search(r"constexpr float kP\[10\] = \{([^}]*)\}", src).group(1)
    return np.array([float(x.strip().rstrip("f")) for x in body.split(",")], dtype=np.float32)


def test_khat_polynomial_is_the_committed_fit_and_matches_arctan():
    """The radiation kernel's atan(x)/x: the coefficients in fft.hip are those
    csrc/fit_atan.py produces, and the kernel's evaluation (polynomial in x^2
    on x <= 1, reflection r (pi/2 - r P(r^2)) above; reciprocal and reciprocal
    square root emulated correctly rounded) agrees with numpy's arctan in FP64
    to 3e-7 relative from x = 0 to 1e4."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "fit_atan", os.path.join(ROOT, "paper_2109_10375_amd", "csrc", "fit_atan.py"))
    fit = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fit)
    kp = _kernel_poly_from_source()
    assert np.array_equal(kp, fit.coefficients_f32()[::-1])
    assert kp[-1] == np.float32(1.0)
    x = np.concatenate([[0.0], np.geomspace(1e-6, 1e4, 400001)])
    x2 = (x * x).astype(np.float32)
    big = x2 > 1
    t = np.where(big, (1.0 / np.where(big, x2, 1).astype(np.float64)).astype(np.float32), x2)
    p = fit.horner_f32(kp[::-1], t).astype(np.float32)
    r = (1.0 / np.sqrt(np.where(big, x2, 1).astype(np.float64))).astype(np.float32)
    g_big = (r * (np.float32(np.pi / 2) - (r * p).astype(np.float32))).astype(np.float32)
    g = np.where(big, g_big, p).astype(np.float64)
    x64 = np.sqrt(x2.astype(np.float64))
    ref = np.ones_like(x64)
    nz = x64 > 0
    ref[nz] = np.arctan(x64[nz]) / x64[nz]
    rel = np.max(np.abs(g - ref) / ref)
    assert rel < 3e-7, rel

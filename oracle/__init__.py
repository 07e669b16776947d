"""FP64 CPU oracle for the AMBER reionization-redshift hot path (test infrastructure).

This package is the checker, not the product: only ``tests/``, the package smoke
check and the benchmark's CPU-baseline leg import it.  It wraps the plain C
definitions in ``amber_oracle.c`` (built with gcc, ``-ffp-contract=off``) and
shares no code with the GPU library.

Paper: Trac et al., "AMBER: A Semi-numerical Abundance Matching Box for the Epoch
of Reionization", arXiv:2109.10375.  Each wrapper names the passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amber_oracle.c")
# AMBER_ORACLE_LIB selects another build of the same source (the sanitizer run)
_LIB = os.environ.get("AMBER_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OK = 0
E_ARG = -1
E_HISTORY = -3
E_DATA = -7
E_RANGE = -8

CONTRACT = 1
EXACT = 0


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d, i, i64, p = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        pd = ctypes.POINTER(ctypes.c_double)
        pi64 = ctypes.POINTER(ctypes.c_int64)
        L.oracle_history_points.argtypes = [d, d, d, pd, pd]
        L.oracle_weibull_x.argtypes = [d, d, d, d]
        L.oracle_weibull_x.restype = d
        L.oracle_weibull_z.argtypes = [d, d, d, d]
        L.oracle_weibull_z.restype = d
        L.oracle_weibull_fit.argtypes = [d, d, d, d, d, d, pd, pd, pd]
        L.oracle_table_geometry.argtypes = [d, d, d, pd, pi64, pd]
        L.oracle_table.argtypes = [d, d, d, d, i64, p]
        L.oracle_kernel_hat.argtypes = [d, d]
        L.oracle_kernel_hat.restype = d
        L.oracle_dft3.argtypes = [i, p, p, i]
        L.oracle_radiation.argtypes = [i, d, p, d, p, pd]
        L.oracle_kernel_real.argtypes = [i, d, d, p]
        L.oracle_direct_convolution.argtypes = [i, d, p, d, p]
        L.oracle_dft_coeff_f32.argtypes = [i, p, i, i, i, pd, pd]
        L.oracle_spectra.argtypes = [i, d, p, i, p, i, i, p, p, p, p, p]
        L.oracle_radiation_from_halos.argtypes = [i, d, i64, p, p, i, i, d, p]
        L.oracle_deposit.argtypes = [i, d, i64, p, p, i, d, p]
        L.oracle_growth.argtypes = [d, d]
        L.oracle_growth.restype = d
        L.oracle_growth_table.argtypes = [d, d, i64, d, d, p]
        L.oracle_zre_growth_f32.argtypes = [i64, p, p, d, d, i64, d, p, p, p, p, i64, p, p, p]
        L.oracle_gauss_legendre.argtypes = [i, p, p]
        L.oracle_rank_f32.argtypes = [i64, p, p]
        L.oracle_rank_f64.argtypes = [i64, p, p]
        L.oracle_mass_fraction.argtypes = [i64, p, p, p]
        L.oracle_zre_f32.argtypes = [i64, p, p, d, d, d, d, i64, d, p, i, p, p, p]
        L.oracle_zre_f64.argtypes = [i64, p, p, d, d, d, d, i64, d, p, i, p, p, p]
        L.oracle_zre_cells_f32.argtypes = [i64, p, p, i64, p, d, d, d, d, i64, d, p, i, p, p]
        L.oracle_invert.argtypes = [i64, p, d, d, d, d, i64, d, p, i, p]
        L.oracle_u128_to_double.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_u128_to_double.restype = d
        L.oracle_num_threads.restype = i
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise OracleError(rc, what)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return lib().oracle_num_threads()


# ---------------------------------------------------------------- history ----

def history_points(z_mid: float, delta_z: float, a_z: float) -> tuple[float, float]:
    """Sec. 3.1.1, Eqs. (zear), (zlat), reading z_lat = z_ear - Delta_z."""
    ze, zl = ctypes.c_double(), ctypes.c_double()
    _check(lib().oracle_history_points(z_mid, delta_z, a_z, ctypes.byref(ze), ctypes.byref(zl)),
           "history_points")
    return ze.value, zl.value


def weibull_x(z, a, b, c):
    """Sec. 3.1.2, Eq. (weibull)."""
    f = lib().oracle_weibull_x
    return np.vectorize(lambda t: f(float(t), a, b, c))(z)


def weibull_z(x, a, b, c):
    """Sec. 3.1.2, inverse of Eq. (weibull)."""
    f = lib().oracle_weibull_z
    return np.vectorize(lambda t: f(float(t), a, b, c))(x)


def weibull_fit(z_mid, delta_z, a_z, x_ear=0.0, x_mid=0.0, x_lat=0.0) -> tuple[float, float, float]:
    """Appendix A: secant solve of f(c_w) = 0, then algebraic a_w, b_w."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().oracle_weibull_fit(z_mid, delta_z, a_z, x_ear, x_mid, x_lat,
                                    ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "weibull_fit")
    return a.value, b.value, c.value


def table_geometry(a, b, c) -> tuple[float, int, float]:
    """Contract-mode table geometry (h, T, z_top); see amber_oracle.c."""
    h, T, zt = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().oracle_table_geometry(a, b, c, ctypes.byref(h), ctypes.byref(T), ctypes.byref(zt)),
           "table_geometry")
    return h.value, T.value, zt.value


def table(a, b, c, h, T) -> np.ndarray:
    X = np.empty(T + 1, dtype=np.float64)
    _check(lib().oracle_table(a, b, c, h, T, _ptr(X)), "table")
    return X


class History:
    """A fitted history: Weibull coefficients plus the contract table."""

    def __init__(self, a, b, c):
        self.a, self.b, self.c = float(a), float(b), float(c)
        self.h, self.T, self.z_top = table_geometry(self.a, self.b, self.c)
        self._X = None

    @classmethod
    def from_params(cls, z_mid, delta_z, a_z, x_ear=0.0, x_mid=0.0, x_lat=0.0):
        return cls(*weibull_fit(z_mid, delta_z, a_z, x_ear, x_mid, x_lat))

    @property
    def X(self) -> np.ndarray:
        if self._X is None:
            self._X = table(self.a, self.b, self.c, self.h, self.T)
        return self._X


# -------------------------------------------------------------- radiation ----

def kernel_hat(k: float, l_mfp: float) -> float:
    """atan(k l)/k, the transform of exp(-r/l)/(4 pi r^2) (Sec. 3.4.1, Eq. intensity)."""
    return lib().oracle_kernel_hat(float(k), float(l_mfp))


def dft3(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Naive separable 3D DFT (unnormalised)."""
    n = x.shape[0]
    re = np.ascontiguousarray(x.real, dtype=np.float64).copy()
    im = np.ascontiguousarray(np.imag(x), dtype=np.float64).copy()
    _check(lib().oracle_dft3(n, _ptr(re), _ptr(im), sign), "dft3")
    return re + 1j * im


def radiation(src: np.ndarray, box_len: float, l_mfp: float, return_imag: bool = False):
    """J = IDFT[DFT(S) Khat] / N^3 in FP64 (Sec. 3.4.1)."""
    n = src.shape[0]
    s = np.ascontiguousarray(src, dtype=np.float64)
    J = np.empty_like(s)
    im = ctypes.c_double()
    _check(lib().oracle_radiation(n, float(box_len), _ptr(s), float(l_mfp), _ptr(J), ctypes.byref(im)),
           "radiation")
    return (J, im.value) if return_imag else J


def kernel_real(n: int, box_len: float, l_mfp: float) -> np.ndarray:
    g = np.empty((n, n, n), dtype=np.float64)
    _check(lib().oracle_kernel_real(n, float(box_len), float(l_mfp), _ptr(g)), "kernel_real")
    return g


def direct_convolution(src: np.ndarray, box_len: float, l_mfp: float) -> np.ndarray:
    n = src.shape[0]
    s = np.ascontiguousarray(src, dtype=np.float64)
    J = np.empty_like(s)
    _check(lib().oracle_direct_convolution(n, float(box_len), _ptr(s), float(l_mfp), _ptr(J)),
           "direct_convolution")
    return J


def dft_coeff(field: np.ndarray, m: tuple[int, int, int]) -> complex:
    """One DFT coefficient of an FP32 field, O(N^3)."""
    f = np.ascontiguousarray(field, dtype=np.float32)
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(lib().oracle_dft_coeff_f32(f.shape[0], _ptr(f), int(m[0]), int(m[1]), int(m[2]),
                                      ctypes.byref(re), ctypes.byref(im)), "dft_coeff")
    return complex(re.value, im.value)


NGP, CIC, TSC = 1, 2, 3


def deposit(n: int, box_len: float, pos: np.ndarray, mass: np.ndarray, p: int, shift: float = 0.0) -> np.ndarray:
    """Mass assignment of a halo catalogue (positions (n_halo, 3) in [0, L))
    to an n^3 mesh with window order p (reading A1), positions shifted by
    ``shift`` cells."""
    ps = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1)
    ms = np.ascontiguousarray(mass, dtype=np.float32)
    mesh = np.empty((n, n, n), dtype=np.float64)
    _check(lib().oracle_deposit(n, float(box_len), ms.size, _ptr(ps), _ptr(ms), int(p), float(shift), _ptr(mesh)),
           "deposit")
    return mesh


def radiation_from_halos(n: int, box_len: float, pos: np.ndarray, mass: np.ndarray, p: int, interlace: bool,
                         l_mfp: float) -> np.ndarray:
    """J of a halo catalogue: interlaced, deconvolved mass assignment (Sec.
    3.2.1, Eqs. interlace, Wofk; readings A1, A2) convolved with the radiation
    kernel (Sec. 3.4.1)."""
    ps = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1)
    ms = np.ascontiguousarray(mass, dtype=np.float32)
    J = np.empty((n, n, n), dtype=np.float64)
    _check(lib().oracle_radiation_from_halos(n, float(box_len), ms.size, _ptr(ps), _ptr(ms), int(p),
                                             1 if interlace else 0, float(l_mfp), _ptr(J)), "radiation_from_halos")
    return J


OMEGA_M = 0.3   # the paper's cosmology (Sec. 2)


def growth(z: float, omega_m: float = OMEGA_M) -> float:
    """Linear growth factor D(z) of flat Lambda-CDM, D -> a early (reading G1)."""
    return float(lib().oracle_growth(float(z), float(omega_m)))


def growth_table(H: "History", z_mid: float, omega_m: float = OMEGA_M) -> np.ndarray:
    """G_j = D(z_j)/D(z_mid) at the inversion-table nodes of history H."""
    G = np.empty(H.T + 1, dtype=np.float64)
    _check(lib().oracle_growth_table(H.a, H.h, H.T, float(z_mid), float(omega_m), _ptr(G)), "growth_table")
    return G


def gauss_legendre(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Nodes and weights of the n-point Gauss-Legendre rule on [-1, 1]."""
    x = np.empty(n)
    w = np.empty(n)
    _check(lib().oracle_gauss_legendre(int(n), _ptr(x), _ptr(w)), "gauss_legendre")
    return x, w


def zre_growth(J: np.ndarray, w: np.ndarray, H: "History", G: np.ndarray, ranks=None):
    """Growth-rescaled abundance matching (Sec. 3.4.2 with the growth factor,
    readings G1, G2): returns (z_re FP32, z_re FP64).  With ``ranks`` (rank
    positions, 0 = brightest) only those ranks are matched and the result is
    (z FP32 per rank, cell index per rank)."""
    j = np.ascontiguousarray(J, dtype=np.float32).reshape(-1)
    ww = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
    Gc = np.ascontiguousarray(G, dtype=np.float64)
    if Gc.size != H.T + 1:
        raise ValueError("growth table must have T + 1 entries")
    if ranks is not None:
        sel = np.ascontiguousarray(np.asarray(ranks, dtype=np.int64).reshape(-1))
        zs = np.empty(sel.size, dtype=np.float32)
        cells = np.empty(sel.size, dtype=np.uint32)
        _check(lib().oracle_zre_growth_f32(j.size, _ptr(j), _ptr(ww), H.a, H.h, H.T, H.z_top, _ptr(H.X), _ptr(Gc),
                                           None, None, sel.size, _ptr(sel), _ptr(zs), _ptr(cells)), "zre_growth")
        return zs, cells
    z32 = np.empty(j.size, dtype=np.float32)
    z64 = np.empty(j.size, dtype=np.float64)
    _check(lib().oracle_zre_growth_f32(j.size, _ptr(j), _ptr(ww), H.a, H.h, H.T, H.z_top, _ptr(H.X), _ptr(Gc),
                                       _ptr(z32), _ptr(z64), 0, None, None, None), "zre_growth")
    return z32.reshape(J.shape), z64.reshape(J.shape)


FIELD_RAW, FIELD_OVERDENSITY, FIELD_REDSHIFT = 0, 1, 2


def spectra(a: np.ndarray, b: np.ndarray | None, box_len: float, n_bins: int, kind_a: int = FIELD_RAW,
            kind_b: int | None = None) -> dict:
    """Shell-averaged auto and cross power spectra (Sec. 2.3, Eqs. Pk, Dk,
    bias, rcc; readings D1, D2), with Delta^2, b_ab and r_ab derived."""
    n = a.shape[0]
    a64 = np.ascontiguousarray(a, dtype=np.float64)
    b64 = a64 if b is None else np.ascontiguousarray(b, dtype=np.float64)
    kb = kind_a if kind_b is None else kind_b
    out = {name: np.zeros(n_bins) for name in ("k", "modes", "p_aa", "p_bb", "p_ab")}
    _check(lib().oracle_spectra(n, float(box_len), _ptr(a64), int(kind_a), _ptr(b64), int(kb), int(n_bins),
                                *[_ptr(out[x]) for x in ("k", "modes", "p_aa", "p_bb", "p_ab")]), "spectra")
    with np.errstate(divide="ignore", invalid="ignore"):
        out["delta2_aa"] = out["k"] ** 3 / (2 * np.pi ** 2) * out["p_aa"]
        out["bias"] = np.sqrt(out["p_aa"] / out["p_bb"])
        out["r"] = out["p_ab"] / np.sqrt(out["p_aa"] * out["p_bb"])
    return out


# ---------------------------------------------------------- abundance match --

def rank(J: np.ndarray) -> np.ndarray:
    """Descending rank order, ties by ascending cell index (Sec. 3.4.2, reading Z3)."""
    flat = np.ascontiguousarray(J).reshape(-1)
    perm = np.empty(flat.size, dtype=np.uint32)
    if flat.dtype == np.float32:
        rc = lib().oracle_rank_f32(flat.size, _ptr(flat), _ptr(perm))
    else:
        flat = flat.astype(np.float64, copy=False)
        rc = lib().oracle_rank_f64(flat.size, _ptr(flat), _ptr(perm))
    _check(rc, "rank")
    return perm


def mass_fraction(perm: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Exact cumulative mass fraction in rank order (Sec. 3.4.2, reading Z4)."""
    p = np.ascontiguousarray(perm, dtype=np.uint32).reshape(-1)
    wf = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
    F = np.empty(p.size, dtype=np.float64)
    _check(lib().oracle_mass_fraction(p.size, _ptr(p), _ptr(wf), _ptr(F)), "mass_fraction")
    return F


def zre(J: np.ndarray, w: np.ndarray, hist: History, mode: int = CONTRACT,
        want_perm: bool = False):
    """Abundance match (Sec. 3.4.2): returns (z_re float32, z_re float64[, perm])."""
    shape = J.shape
    flat = np.ascontiguousarray(J).reshape(-1)
    wf = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
    n = flat.size
    z32 = np.empty(n, dtype=np.float32)
    z64 = np.empty(n, dtype=np.float64)
    perm = np.empty(n, dtype=np.uint32)
    X = hist.X if mode == CONTRACT else np.zeros(2)
    args = (hist.a, hist.b, hist.c, hist.h, hist.T, hist.z_top, _ptr(X), mode, _ptr(z32), _ptr(z64), _ptr(perm))
    if flat.dtype == np.float32:
        rc = lib().oracle_zre_f32(n, _ptr(flat), _ptr(wf), *args)
    else:
        flat = flat.astype(np.float64, copy=False)
        rc = lib().oracle_zre_f64(n, _ptr(flat), _ptr(wf), *args)
    _check(rc, "zre")
    out = (z32.reshape(shape), z64.reshape(shape))
    return out + (perm,) if want_perm else out


def zre_cells(J: np.ndarray, w: np.ndarray, cells, hist: History, mode: int = CONTRACT):
    """z_re of selected cells, one by one in O(N) each; returns (z float32, F float64)."""
    flat = np.ascontiguousarray(J, dtype=np.float32).reshape(-1)
    wf = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
    c = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
    z = np.empty(c.size, dtype=np.float32)
    F = np.empty(c.size, dtype=np.float64)
    X = hist.X if mode == CONTRACT else np.zeros(2)
    _check(lib().oracle_zre_cells_f32(flat.size, _ptr(flat), _ptr(wf), c.size, _ptr(c),
                                      hist.a, hist.b, hist.c, hist.h, hist.T, hist.z_top,
                                      _ptr(X), mode, _ptr(z), _ptr(F)), "zre_cells")
    return z, F


def invert(F, hist: History, mode: int = CONTRACT) -> np.ndarray:
    """z = x_i^{-1}(F): closed form (exact mode) or table interpolation (contract)."""
    f = np.ascontiguousarray(F, dtype=np.float64).reshape(-1)
    z = np.empty_like(f)
    X = hist.X if mode == CONTRACT else np.zeros(2)
    _check(lib().oracle_invert(f.size, _ptr(f), hist.a, hist.b, hist.c, hist.h, hist.T, hist.z_top,
                               _ptr(X), mode, _ptr(z)), "invert")
    return z


def u128_to_double(v: int) -> float:
    return lib().oracle_u128_to_double((v >> 64) & ((1 << 64) - 1), v & ((1 << 64) - 1))


def zre_per_cell_check(J32: np.ndarray, J64: np.ndarray, w: np.ndarray, hist: History, z_gpu: np.ndarray,
                       tol: float = 1e-4) -> dict:
    """End-to-end check of a z_re field matched from an FP32 intensity field
    J32 (Sec. 3.4.2), cell by cell, against the FP64 oracle:

      1. every cell is within ``tol`` of the exact-mode match of the same FP32
         field (rank order of J32, exact cumulative mass, closed-form
         inversion): the matching itself is right in every cell;
      2. against the exact-mode match of the FP64 field J64, a cell can differ
         by more than ``tol`` only where its exact ionized-mass fraction F
         differs between the two rank orders (the FP32 field orders some
         nearly equal intensities differently); such cells are counted.

    Raises AssertionError naming the first failing cell; returns statistics."""
    shape = J32.shape
    wf = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
    zg = np.asarray(z_gpu, dtype=np.float64).reshape(-1)
    _, z32x = zre(np.ascontiguousarray(J32, dtype=np.float32), wf.reshape(shape), hist, mode=EXACT)
    err32 = np.abs(zg - z32x.reshape(-1))
    bad = np.nonzero(err32 > tol)[0]
    assert bad.size == 0, (f"cell {int(bad[0])}: z {zg[bad[0]]!r} vs exact match of the same FP32 field "
                           f"{z32x.reshape(-1)[bad[0]]!r} ({bad.size} cells beyond {tol})")
    _, z64x = zre(np.ascontiguousarray(J64, dtype=np.float64), wf.reshape(shape), hist, mode=EXACT)
    err64 = np.abs(zg - z64x.reshape(-1))
    pg = rank(np.ascontiguousarray(J32, dtype=np.float32))
    po = rank(np.ascontiguousarray(J64, dtype=np.float64))
    Fg = np.empty(pg.size)
    Fo = np.empty(po.size)
    Fg[pg] = mass_fraction(pg, wf)
    Fo[po] = mass_fraction(po, wf)
    over = err64 > tol
    unexplained = np.nonzero(over & (Fg == Fo))[0]
    assert unexplained.size == 0, (f"cell {int(unexplained[0])}: beyond {tol} of the FP64 match with the "
                                   f"same ionized-mass fraction in both orders")
    pos_g = np.empty_like(pg)
    pos_g[pg] = np.arange(pg.size, dtype=np.uint32)
    pos_o = np.empty_like(po)
    pos_o[po] = np.arange(po.size, dtype=np.uint32)
    disp = np.abs(pos_g.astype(np.int64) - pos_o.astype(np.int64))
    return {"max_err_same_field": float(err32.max()), "frac_within_tol_fp64": float(np.mean(~over)),
            "cells_over_tol_fp64": int(over.sum()), "max_err_fp64": float(err64.max()),
            "max_rank_displacement": int(disp.max()), "cells_moved": int(np.sum(disp > 0))}

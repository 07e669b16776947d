"""ctypes binding of libamber.so (argument marshalling only).

Every method maps onto one C-ABI entry point of ``include/amber.h`` with the
same name; tensors must already live on the GPU, and work is enqueued on
torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libamber.so")

OK = 0
E_ARG, E_SIZE, E_HISTORY, E_WORKSPACE, E_HIP, E_UNIMPL = -1, -2, -3, -4, -5, -6
STATUS_NAN_J, STATUS_BAD_W, STATUS_RANGE = 1, 2, 4

SYMBOLS = [
    "amber_version", "amber_strerror", "amber_weibull_fit", "amber_weibull_from_coeffs",
    "amber_weibull_table", "amber_plan_create", "amber_plan_destroy", "amber_workspace_bytes",
    "amber_radiation", "amber_rank", "amber_zre", "amber_status", "amber_profile_begin",
    "amber_profile_end", "amber_batch_workspace_bytes", "amber_batch_run", "amber_spectra_workspace_bytes",
    "amber_spectra", "amber_growth_table", "amber_halo_workspace_bytes", "amber_radiation_from_halos",
    "amber_fft_schedules", "amber_fft_schedule_info", "amber_plan_set_schedule", "amber_plan_get_schedule",
    "amber_plan_tune", "amber_history_prepare", "amber_growth_prepare", "amber_zre_noalloc",
    "amber_executor_create", "amber_executor_destroy",
]
NOALLOC_MAX_N = 128
NOALLOC_SCRATCH_BYTES = 68 << 20
ASSIGN_NGP, ASSIGN_CIC, ASSIGN_TSC = 1, 2, 3
FIELD_RAW, FIELD_OVERDENSITY, FIELD_REDSHIFT = 0, 1, 2


class AmberWeibull(ctypes.Structure):
    _fields_ = [("a_w", ctypes.c_double), ("b_w", ctypes.c_double), ("c_w", ctypes.c_double),
                ("h", ctypes.c_double), ("z_top", ctypes.c_double), ("table_n", ctypes.c_int64),
                ("d_table", ctypes.c_void_p), ("d_growth", ctypes.c_void_p)]


class AmberKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double)]


class AmberHistory(ctypes.Structure):
    _fields_ = [("z_mid", ctypes.c_double), ("delta_z", ctypes.c_double), ("a_z", ctypes.c_double),
                ("x_ear", ctypes.c_double), ("x_mid", ctypes.c_double), ("x_lat", ctypes.c_double)]


class AmberBatchItem(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("d_src", ctypes.c_void_p), ("d_w", ctypes.c_void_p),
                ("n_lmfp", ctypes.c_int), ("l_mfp", ctypes.POINTER(ctypes.c_double)),
                ("d_J", ctypes.POINTER(ctypes.c_void_p)), ("n_hist", ctypes.c_int),
                ("hist", ctypes.POINTER(AmberWeibull)), ("d_zre", ctypes.POINTER(ctypes.c_void_p))]


class AmberError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib().amber_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(_LIB_PATH)
        vp, sz, i, d, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double, ctypes.c_int64
        L.amber_version.restype = ctypes.c_char_p
        L.amber_strerror.restype = ctypes.c_char_p
        L.amber_strerror.argtypes = [i]
        L.amber_weibull_fit.argtypes = [ctypes.POINTER(AmberHistory), ctypes.POINTER(AmberWeibull)]
        L.amber_weibull_from_coeffs.argtypes = [d, d, d, ctypes.POINTER(AmberWeibull)]
        L.amber_weibull_table.argtypes = [ctypes.POINTER(AmberWeibull), vp, i64]
        L.amber_growth_table.argtypes = [ctypes.POINTER(AmberWeibull), d, d, vp, i64]
        L.amber_halo_workspace_bytes.argtypes = [vp]
        L.amber_halo_workspace_bytes.restype = sz
        L.amber_radiation_from_halos.argtypes = [vp, vp, vp, i64, i, i, ctypes.POINTER(d), i, ctypes.POINTER(vp), vp,
                                                 sz, vp]
        L.amber_plan_create.argtypes = [ctypes.POINTER(vp), i, d]
        L.amber_plan_destroy.argtypes = [vp]
        L.amber_plan_destroy.restype = None
        L.amber_workspace_bytes.argtypes = [vp, i, i]
        L.amber_workspace_bytes.restype = sz
        L.amber_radiation.argtypes = [vp, vp, ctypes.POINTER(d), i, ctypes.POINTER(vp), vp, sz, vp]
        L.amber_rank.argtypes = [vp, vp, vp, vp, sz, vp]
        L.amber_zre.argtypes = [vp, vp, vp, ctypes.POINTER(AmberWeibull), i, ctypes.POINTER(vp), vp, sz, vp]
        L.amber_zre_noalloc.argtypes = [vp, vp, vp, ctypes.POINTER(AmberWeibull), i, ctypes.POINTER(vp), vp]
        L.amber_status.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_uint)]
        L.amber_history_prepare.argtypes = [ctypes.POINTER(AmberHistory), ctypes.POINTER(AmberWeibull), vp, sz, vp]
        L.amber_growth_prepare.argtypes = [ctypes.POINTER(AmberWeibull), d, d, vp, sz, vp]
        L.amber_profile_begin.argtypes = [vp, i]
        L.amber_profile_end.argtypes = [vp, ctypes.POINTER(AmberKernelTime), i, ctypes.POINTER(i)]
        L.amber_batch_workspace_bytes.argtypes = [ctypes.POINTER(AmberBatchItem), i, i]
        L.amber_batch_workspace_bytes.restype = sz
        L.amber_batch_run.argtypes = [ctypes.POINTER(AmberBatchItem), i, vp, vp, sz, vp, vp]
        L.amber_executor_create.argtypes = [ctypes.POINTER(vp), i]
        L.amber_executor_destroy.argtypes = [vp]
        L.amber_executor_destroy.restype = None
        L.amber_spectra_workspace_bytes.argtypes = [vp]
        L.amber_spectra_workspace_bytes.restype = sz
        L.amber_spectra.argtypes = [vp, vp, i, vp, i, i, vp, vp, sz, vp]
        ip = ctypes.POINTER(i)
        L.amber_fft_schedules.argtypes = [i, ip, ip]
        L.amber_fft_schedule_info.argtypes = [i, i, i, ip, ip]
        L.amber_plan_set_schedule.argtypes = [vp, i, i]
        L.amber_plan_get_schedule.argtypes = [vp, ip, ip]
        L.amber_plan_tune.argtypes = [vp, vp, vp, vp, sz, i, ctypes.POINTER(ctypes.c_float), ip, ip, vp]
        _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise AmberError(rc, what)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype: torch.dtype, numel: int, what: str) -> ctypes.c_void_p:
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{what}: expected a contiguous CUDA {dtype} tensor of {numel} elements")
    return ctypes.c_void_p(t.data_ptr())


class History:
    """A reionization history (Sec. 3.1): Weibull coefficients + device table."""

    def __init__(self, w: AmberWeibull, device=None):
        self.w = w
        host = torch.empty(w.table_n, dtype=torch.float64)
        _check(lib().amber_weibull_table(ctypes.byref(w), ctypes.c_void_p(host.data_ptr()), w.table_n),
               "amber_weibull_table")
        self.table = host.to(device or torch.device("cuda"))
        self.w.d_table = self.table.data_ptr()

    @classmethod
    def from_params(cls, z_mid, delta_z, a_z, x_ear=0.0, x_mid=0.0, x_lat=0.0, device=None):
        """amber_history_prepare: the fit and its device table in one call."""
        h = AmberHistory(z_mid, delta_z, a_z, x_ear, x_mid, x_lat)
        w = AmberWeibull()
        _check(lib().amber_history_prepare(ctypes.byref(h), ctypes.byref(w), None, 0, None), "amber_history_prepare")
        table = torch.empty(w.table_n, dtype=torch.float64, device=device or torch.device("cuda"))
        _check(lib().amber_history_prepare(ctypes.byref(h), ctypes.byref(w), ctypes.c_void_p(table.data_ptr()),
                                           table.numel() * 8, _stream()), "amber_history_prepare")
        obj = cls.__new__(cls)
        obj.w = w
        obj.table = table
        return obj

    @classmethod
    def from_coeffs(cls, a_w, b_w, c_w, device=None):
        w = AmberWeibull()
        _check(lib().amber_weibull_from_coeffs(a_w, b_w, c_w, ctypes.byref(w)), "amber_weibull_from_coeffs")
        return cls(w, device)

    @staticmethod
    def fit_host(z_mid, delta_z, a_z, x_ear=0.0, x_mid=0.0, x_lat=0.0) -> AmberWeibull:
        """The library's host-side fit without touching the GPU."""
        h = AmberHistory(z_mid, delta_z, a_z, x_ear, x_mid, x_lat)
        w = AmberWeibull()
        _check(lib().amber_weibull_fit(ctypes.byref(h), ctypes.byref(w)), "amber_weibull_fit")
        return w

    @property
    def coeffs(self):
        return self.w.a_w, self.w.b_w, self.w.c_w

    def with_growth(self, z_mid: float, omega_m: float = 0.3) -> "History":
        """The same history matched with growth-rescaled overdensities
        (amber_growth_table: pairs (X_j, G_j = D(z_j)/D(z_mid)) on the device)."""
        w = AmberWeibull.from_buffer_copy(self.w)
        h = History.__new__(History)
        h.w = w
        h.table = self.table
        h.growth = torch.empty(2 * w.table_n, dtype=torch.float64, device=self.table.device)
        h.w.d_table = self.table.data_ptr()
        _check(lib().amber_growth_prepare(ctypes.byref(h.w), float(z_mid), float(omega_m),
                                          ctypes.c_void_p(h.growth.data_ptr()), h.growth.numel() * 8, _stream()),
               "amber_growth_prepare")
        return h

    def with_growth_pairs(self, pairs: torch.Tensor) -> "History":
        """The same history matched with a caller-built growth table: a
        contiguous CUDA float64 tensor of 2 table_n values, the pairs
        (X_j, G_j) that amber_weibull.d_growth points to."""
        _dev_ptr(pairs, torch.float64, 2 * self.w.table_n, "growth pairs")
        if pairs.data_ptr() % 16:
            raise ValueError("growth pairs: the device table must be 16-byte aligned")
        w = AmberWeibull.from_buffer_copy(self.w)
        h = History.__new__(History)
        h.w = w
        h.table = self.table
        h.growth = pairs
        h.w.d_table = self.table.data_ptr()
        h.w.d_growth = pairs.data_ptr()
        return h

    @staticmethod
    def growth_table_host(w: AmberWeibull, z_mid: float, omega_m: float = 0.3) -> torch.Tensor:
        """The library's host growth table for a fitted history (no GPU work):
        pairs (X_j, G_j), 2 table_n doubles."""
        host = torch.empty(2 * w.table_n, dtype=torch.float64)
        _check(lib().amber_growth_table(ctypes.byref(w), float(z_mid), float(omega_m),
                                        ctypes.c_void_p(host.data_ptr()), w.table_n), "amber_growth_table")
        return host


def fft_schedules(n: int) -> dict:
    """amber_fft_schedules + amber_fft_schedule_info: the compiled FFT launch
    candidates for grid size n, {"col": [(N1, C), ...], "z": [(M1, ZL), ...]}
    (index 0 is the default).  Host only."""
    nc, nz = ctypes.c_int(), ctypes.c_int()
    _check(lib().amber_fft_schedules(int(n), ctypes.byref(nc), ctypes.byref(nz)), "amber_fft_schedules")
    out = {"col": [], "z": []}
    for kind, key, count in ((0, "col", nc.value), (1, "z", nz.value)):
        for idx in range(count):
            a, b = ctypes.c_int(), ctypes.c_int()
            _check(lib().amber_fft_schedule_info(int(n), kind, idx, ctypes.byref(a), ctypes.byref(b)),
                   "amber_fft_schedule_info")
            out[key].append((a.value, b.value))
    return out


class Plan:
    """An N^3 periodic box of side box_len on the current GPU (amber_plan_create)."""

    def __init__(self, n: int, box_len: float):
        self.n = int(n)
        self.box_len = float(box_len)
        self.n3 = self.n ** 3
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        _check(lib().amber_plan_create(ctypes.byref(h), self.n, self.box_len), "amber_plan_create")
        self._h = h
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.amber_plan_destroy(h)
            self._h = None

    def workspace_bytes(self, n_lmfp: int = 1, n_hist: int = 1) -> int:
        return int(lib().amber_workspace_bytes(self._h, int(n_lmfp), int(n_hist)))

    def workspace(self, n_lmfp: int = 1) -> torch.Tensor:
        need = self.workspace_bytes(n_lmfp)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            torch.cuda.empty_cache()
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def radiation(self, S: torch.Tensor, l_mfp: Sequence[float], out: Sequence[torch.Tensor] | None = None):
        """amber_radiation: one J field per mean free path."""
        l = [float(x) for x in l_mfp]
        if out is None:
            out = [torch.empty((self.n,) * 3, dtype=torch.float32, device=self.device) for _ in l]
        src = _dev_ptr(S, torch.float32, self.n3, "S")
        ptrs = (ctypes.c_void_p * len(l))(*[_dev_ptr(o, torch.float32, self.n3, "J").value for o in out])
        larr = (ctypes.c_double * len(l))(*l)
        ws = self.workspace(len(l))
        _check(lib().amber_radiation(self._h, src, larr, len(l), ptrs, ctypes.c_void_p(ws.data_ptr()),
                                     ws.numel(), _stream()), "amber_radiation")
        return list(out)

    def radiation_from_halos(self, pos: torch.Tensor, mass: torch.Tensor, l_mfp: Sequence[float],
                             scheme: int = ASSIGN_CIC, interlace: bool = True,
                             out: Sequence[torch.Tensor] | None = None):
        """amber_radiation_from_halos: J per mean free path from a halo
        catalogue (positions (n_halo, 3) in [0, box_len), masses (n_halo,))."""
        l = [float(x) for x in l_mfp]
        nh = int(mass.numel())
        if out is None:
            out = [torch.empty((self.n,) * 3, dtype=torch.float32, device=self.device) for _ in l]
        pp = _dev_ptr(pos, torch.float32, 3 * nh, "pos") if nh else None
        pm = _dev_ptr(mass, torch.float32, nh, "mass") if nh else None
        ptrs = (ctypes.c_void_p * len(l))(*[_dev_ptr(o, torch.float32, self.n3, "J").value for o in out])
        larr = (ctypes.c_double * len(l))(*l)
        need = int(lib().amber_halo_workspace_bytes(self._h))
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        _check(lib().amber_radiation_from_halos(self._h, pp, pm, nh, int(scheme), 1 if interlace else 0, larr, len(l),
                                                ptrs, ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                                _stream()), "amber_radiation_from_halos")
        return list(out)

    def rank(self, J: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """amber_rank: the descending rank order (uint32 stored in an int32 tensor)."""
        if out is None:
            out = torch.empty(self.n3, dtype=torch.int32, device=self.device)
        ws = self.workspace(1)
        _check(lib().amber_rank(self._h, _dev_ptr(J, torch.float32, self.n3, "J"),
                                _dev_ptr(out, torch.int32, self.n3, "perm"), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel(), _stream()), "amber_rank")
        return out

    def zre(self, J: torch.Tensor, w: torch.Tensor, hists: Sequence[History],
            out: Sequence[torch.Tensor] | None = None):
        """amber_zre: one z_re field per history."""
        if out is None:
            out = [torch.empty((self.n,) * 3, dtype=torch.float32, device=self.device) for _ in hists]
        harr = (AmberWeibull * len(hists))(*[h.w for h in hists])
        ptrs = (ctypes.c_void_p * len(hists))(*[_dev_ptr(o, torch.float32, self.n3, "z_re").value for o in out])
        ws = self.workspace(1)
        _check(lib().amber_zre(self._h, _dev_ptr(J, torch.float32, self.n3, "J"),
                               _dev_ptr(w, torch.float32, self.n3, "w"), harr, len(hists), ptrs,
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()), "amber_zre")
        return list(out)

    def zre_noalloc(self, J: torch.Tensor, w: torch.Tensor, hists: Sequence[History],
                    out: Sequence[torch.Tensor] | None = None):
        """amber_zre_noalloc: amber_zre with the library's static scratch
        instead of a workspace (N <= 128; nothing is allocated when out is
        given)."""
        if out is None:
            out = [torch.empty((self.n,) * 3, dtype=torch.float32, device=self.device) for _ in hists]
        harr = (AmberWeibull * len(hists))(*[h.w for h in hists])
        ptrs = (ctypes.c_void_p * len(hists))(*[_dev_ptr(o, torch.float32, self.n3, "z_re").value for o in out])
        _check(lib().amber_zre_noalloc(self._h, _dev_ptr(J, torch.float32, self.n3, "J"),
                                       _dev_ptr(w, torch.float32, self.n3, "w"), harr, len(hists), ptrs, _stream()),
               "amber_zre_noalloc")
        return list(out)

    def spectra(self, a: torch.Tensor, b: torch.Tensor | None = None, kind_a: int = FIELD_RAW,
                kind_b: int | None = None, n_bins: int | None = None) -> dict:
        """amber_spectra: shell-averaged k, modes, P_aa, P_bb, P_ab, Delta^2_aa,
        b_ab and r_ab (Sec. 2.3), as float64 tensors on the host."""
        nb = self.n // 2 + 1 if n_bins is None else int(n_bins)
        need = int(lib().amber_spectra_workspace_bytes(self._h))
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        out = torch.empty(8 * nb, dtype=torch.float64, device=self.device)
        pa = _dev_ptr(a, torch.float32, self.n3, "a")
        pb = _dev_ptr(b, torch.float32, self.n3, "b") if b is not None else None
        _check(lib().amber_spectra(self._h, pa, int(kind_a), pb, int(kind_a if kind_b is None else kind_b), nb,
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(self._ws.data_ptr()),
                                   self._ws.numel(), _stream()), "amber_spectra")
        rows = out.view(8, nb).cpu()
        names = ("k", "modes", "p_aa", "p_bb", "p_ab", "delta2_aa", "bias", "r")
        return {name: rows[i] for i, name in enumerate(names)}

    @property
    def schedule(self) -> tuple:
        """amber_plan_get_schedule: (column candidate, z candidate)."""
        c, z = ctypes.c_int(), ctypes.c_int()
        _check(lib().amber_plan_get_schedule(self._h, ctypes.byref(c), ctypes.byref(z)), "amber_plan_get_schedule")
        return (c.value, z.value)

    def set_schedule(self, col: int, z: int) -> None:
        """amber_plan_set_schedule."""
        _check(lib().amber_plan_set_schedule(self._h, int(col), int(z)), "amber_plan_set_schedule")

    def tune(self, S: torch.Tensor, reps: int = 5) -> dict:
        """amber_plan_tune: time every FFT candidate pair on S and keep the
        fastest.  Returns {"col", "z", "ms": [[ms per pass] per z] per col}."""
        cand = fft_schedules(self.n)
        nc, nz = len(cand["col"]), len(cand["z"])
        J = torch.empty((self.n,) * 3, dtype=torch.float32, device=self.device)
        ms = (ctypes.c_float * (nc * nz))()
        c, z = ctypes.c_int(), ctypes.c_int()
        ws = self.workspace(1)
        _check(lib().amber_plan_tune(self._h, _dev_ptr(S, torch.float32, self.n3, "S"),
                                     _dev_ptr(J, torch.float32, self.n3, "J"), ctypes.c_void_p(ws.data_ptr()),
                                     ws.numel(), int(reps), ms, ctypes.byref(c), ctypes.byref(z), _stream()),
               "amber_plan_tune")
        return {"col": c.value, "z": z.value, "ms": [[float(ms[a * nz + b]) for b in range(nz)] for a in range(nc)]}

    def profile_begin(self, capacity: int = 4096) -> None:
        """amber_profile_begin: time every kernel of the following calls."""
        _check(lib().amber_profile_begin(self._h, int(capacity)), "amber_profile_begin")

    def profile_end(self) -> dict:
        """amber_profile_end: {kernel name: (launches, total ms)}."""
        buf = (AmberKernelTime * 64)()
        n = ctypes.c_int()
        _check(lib().amber_profile_end(self._h, buf, 64, ctypes.byref(n)), "amber_profile_end")
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(n.value)}

    def status(self) -> int:
        """amber_status: device status bits of every ranking/matching call on
        this plan since the last amber_status (read and cleared)."""
        v = ctypes.c_uint()
        _check(lib().amber_status(self._h, _stream(), ctypes.byref(v)), "amber_status")
        return int(v.value)


class BatchItem:
    """One box of a batch (amber_batch_item): its fields, mean free paths and
    histories.  z_re of J_l under history h is zre[l][h]; an entry may be None
    (that pair is not matched)."""

    def __init__(self, plan: Plan, S: torch.Tensor | None, w: torch.Tensor, l_mfp: Sequence[float],
                 J: Sequence[torch.Tensor], hists: Sequence[History],
                 zre: Sequence[Sequence[torch.Tensor | None]]):
        nl, nh = len(J), len(hists)
        if S is not None and len(l_mfp) != nl:
            raise ValueError("one J field per mean free path")
        if len(zre) != nl or any(len(row) != nh for row in zre):
            raise ValueError("zre must hold n_lmfp rows of n_hist fields")
        self.plan, self.S, self.w, self.J, self.hists, self.zre = plan, S, w, list(J), list(hists), zre
        n3 = plan.n3
        self._l = (ctypes.c_double * max(1, nl))(*[float(x) for x in l_mfp] if S is not None else [])
        self._J = (ctypes.c_void_p * nl)(*[_dev_ptr(t, torch.float32, n3, "J").value for t in J])
        self._h = (AmberWeibull * nh)(*[h.w for h in hists])
        flat = [z for row in zre for z in row]
        self._z = (ctypes.c_void_p * len(flat))(*[None if t is None else _dev_ptr(t, torch.float32, n3, "z_re").value
                                                  for t in flat])
        self.c = AmberBatchItem(plan._h.value, _dev_ptr(S, torch.float32, n3, "S").value if S is not None else None,
                                _dev_ptr(w, torch.float32, n3, "w").value, nl,
                                ctypes.cast(self._l, ctypes.POINTER(ctypes.c_double)),
                                ctypes.cast(self._J, ctypes.POINTER(ctypes.c_void_p)), nh,
                                ctypes.cast(self._h, ctypes.POINTER(AmberWeibull)),
                                ctypes.cast(self._z, ctypes.POINTER(ctypes.c_void_p)))


class Executor:
    """Side streams and events for running the boxes of a batch concurrently
    (amber_executor_create); lane 0 is the calling stream."""

    def __init__(self, lanes: int):
        h = ctypes.c_void_p()
        _check(lib().amber_executor_create(ctypes.byref(h), int(lanes)), "amber_executor_create")
        self._h = h
        self.lanes = int(lanes)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.amber_executor_destroy(h)
            self._h = None


class Batch:
    """A fixed list of boxes run by amber_batch_run with one workspace (one
    slice per lane)."""

    def __init__(self, items: Sequence[BatchItem], ws: torch.Tensor | None = None, lanes: int = 1):
        self.items = list(items)
        self.lanes = max(1, min(int(lanes), len(self.items)))
        self._arr = (AmberBatchItem * len(self.items))(*[it.c for it in self.items])
        need = int(lib().amber_batch_workspace_bytes(self._arr, len(self.items), self.lanes))
        if need == 0:
            raise ValueError("invalid batch")
        self.device = self.items[0].plan.device
        if ws is not None and (not ws.is_cuda or ws.dtype != torch.uint8 or ws.numel() < need):
            raise ValueError(f"workspace: expected a CUDA uint8 tensor of at least {need} bytes")
        self.ws = ws if ws is not None else torch.empty(need, dtype=torch.uint8, device=self.device)
        self.status = torch.zeros(len(self.items), dtype=torch.int32, device=self.device)
        self.executor = Executor(self.lanes) if self.lanes > 1 else None

    @staticmethod
    def workspace_bytes(items: Sequence[BatchItem], lanes: int = 1) -> int:
        arr = (AmberBatchItem * len(items))(*[it.c for it in items])
        return int(lib().amber_batch_workspace_bytes(arr, len(items), max(1, min(int(lanes), len(items)))))

    def run(self) -> None:
        """amber_batch_run on torch's current stream; per-box status bits land in self.status."""
        ex = self.executor._h if self.executor is not None else None
        _check(lib().amber_batch_run(self._arr, len(self.items), ctypes.c_void_p(self.status.data_ptr()),
                                     ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream(), ex),
               "amber_batch_run")

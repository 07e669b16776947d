"""Seeded synthetic boxes standing in for the paper's LPT/ESF fields.

The paper builds its density with 2LPT + TSC and its source field from an
excursion-set halo mass density (Secs. 3.2-3.3); those need a linear power
spectrum, N-body calibrations and catalogs that are not available.  These
generators reproduce the *structure* the hot path sees:

* density: a Gaussian random field with P(k) proportional to k^-2.5 (P(0) = 0),
  standardised and exponentiated into a lognormal 1+delta of unit mean and unit
  variance (then rescaled to sample mean exactly 1);
* source: halos placed in cells drawn with probability proportional to 1+delta,
  uniform inside the cell, masses from dN/dM proportional to M^-1.9 on
  [M_lo, M_hi], deposited with periodic cloud-in-cell;
* intensity (for matching-only tests): a smooth correlated field with planted
  exact ties, signed zeros and negative values.

Everything is drawn with ``torch.Generator(device).manual_seed(seed)``; the
same seed on the same device type gives the same box.  Work runs on the device
given (CPU for the sizes the oracle handles, the GPU for the large boxes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch


@dataclass(frozen=True)
class BoxConfig:
    name: str
    n: int
    box_len: float               # h^-1 Mpc
    n_halo: int
    m_lo: float                  # h^-1 Msun
    m_hi: float
    l_mfp: tuple = (3.0,)        # h^-1 Mpc
    histories: tuple = ((8.0, 4.0, 3.0),)   # (z_mid, Delta_z, A_z)
    index: int = 0
    notes: str = ""


# The workloads: a 64^3 box the oracle runs end to end, a 256^3 box, a 512^3
# box with an l_mfp x history sweep, and the 1024^3 headline box.
CONFIGS = {
    "c1": BoxConfig("c1", 64, 100.0, 20_000, 1e9, 1e12, index=1,
                    notes="64^3, 100 Mpc/h, 20k halos on [1e9,1e12]"),
    "c2": BoxConfig("c2", 256, 500.0, 1_300_000, 1e10, 1e12, index=2,
                    notes="256^3, 500 Mpc/h, 1.3M halos on [1e10,1e12]"),
    "c3": BoxConfig("c3", 512, 1000.0, 10_000_000, 1e10, 1e12,
                    l_mfp=(0.5, 1.0, 2.0, 3.0, 5.0, 10.0, 20.0, 50.0),
                    histories=((8.0, 4.0, 3.0), (7.95, 4.68, 2.90), (7.91, 5.45, 2.69), (7.83, 6.54, 2.33)),
                    index=3, notes="512^3, 1 Gpc/h, 10M halos, 8 l_mfp x 4 histories"),
    "H": BoxConfig("H", 1024, 2000.0, 80_000_000, 1e10, 1e12, index=6,
                   notes="1024^3, 2 Gpc/h, 80M halos on [1e10,1e12], l_mfp=3, (8,4,3)"),
}


def config_seed(index: int, box: int = 0) -> int:
    return 210910375 + 1000 * index + box


def _gen(device, seed: int) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _int_freq(n: int, device, half: bool = False) -> torch.Tensor:
    if half:
        return torch.arange(n // 2 + 1, device=device, dtype=torch.float64)
    f = torch.arange(n, device=device, dtype=torch.float64)
    return torch.where(f <= n // 2, f, f - n)


def _grf(n: int, slope: float, gen: torch.Generator, device, dtype) -> torch.Tensor:
    """Standardised Gaussian random field with P(k) ~ k^slope, P(0) = 0."""
    white = torch.randn((n, n, n), generator=gen, device=device, dtype=dtype)
    wk = torch.fft.rfftn(white)
    del white
    fx = _int_freq(n, device).to(dtype)
    fz = _int_freq(n, device, half=True).to(dtype)
    amp = torch.empty(wk.shape, device=device, dtype=dtype)
    for ix in range(n):   # plane by plane keeps the temporary small at 1024^3
        k2 = fx[ix] ** 2 + fx[:, None] ** 2 + fz[None, :] ** 2
        a = torch.where(k2 > 0, k2.clamp_min(1e-30) ** (slope / 4.0), torch.zeros_like(k2))
        amp[ix] = a
    wk *= amp
    del amp
    g = torch.fft.irfftn(wk, s=(n, n, n))
    del wk
    g -= g.mean()
    g /= g.std()
    return g


def make_density(n: int, seed: int, device="cpu", dtype=torch.float64) -> torch.Tensor:
    """Lognormal 1+delta of unit mean and unit variance from a k^-2.5 GRF."""
    gen = _gen(device, seed)
    g = _grf(n, -2.5, gen, device, dtype)
    s2 = math.log(2.0)                     # exp(s^2) - 1 = 1  -> unit variance
    w = torch.exp(math.sqrt(s2) * g - 0.5 * s2)
    w /= w.mean()
    return w


def _cic_deposit(n: int, pos: torch.Tensor, mass: torch.Tensor, dtype) -> torch.Tensor:
    """Periodic cloud-in-cell; positions in cell units, cell centres at i + 1/2."""
    d = pos - 0.5
    i0 = torch.floor(d)
    f = (d - i0).to(dtype)
    i0 = i0.to(torch.int64) % n
    i1 = (i0 + 1) % n
    out = torch.zeros(n * n * n, device=pos.device, dtype=dtype)
    m = mass.to(dtype)
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        ix = i1[:, 0] if cx else i0[:, 0]
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            iy = i1[:, 1] if cy else i0[:, 1]
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                iz = i1[:, 2] if cz else i0[:, 2]
                out.index_add_(0, (ix * n + iy) * n + iz, m * wx * wy * wz)
    return out.view(n, n, n)


def make_box(cfg: BoxConfig, box: int = 0, device="cpu", dtype=None, chunk: int = 8_000_000):
    """Return (w, S) as float32 tensors of shape (n, n, n) on ``device``.

    w = 1+delta (gas-mass weights), S = CIC-deposited halo mass (source field).
    """
    n = cfg.n
    if dtype is None:
        dtype = torch.float64 if n <= 256 else torch.float32
    seed = config_seed(cfg.index, box)
    w = make_density(n, seed, device=device, dtype=dtype)
    gen = _gen(device, seed + 7)
    cdf = torch.cumsum(w.reshape(-1).to(torch.float64), 0)
    total = cdf[-1].item()
    a = cfg.m_lo ** -0.9
    b = cfg.m_hi ** -0.9
    S = torch.zeros(n * n * n, device=device, dtype=dtype)
    left = cfg.n_halo
    while left > 0:
        m = min(left, chunk)
        u = torch.rand(m, generator=gen, device=device, dtype=torch.float64) * total
        cell = torch.searchsorted(cdf, u).clamp_max(n * n * n - 1)
        cx = cell // (n * n)
        cy = (cell // n) % n
        cz = cell % n
        off = torch.rand((m, 3), generator=gen, device=device, dtype=torch.float64)
        pos = torch.stack([cx, cy, cz], 1).to(torch.float64) + off
        um = torch.rand(m, generator=gen, device=device, dtype=torch.float64)
        mass = (a + um * (b - a)) ** (-1.0 / 0.9)
        S += _cic_deposit(n, pos, mass, dtype).reshape(-1)
        left -= m
        del u, cell, cx, cy, cz, off, pos, um, mass
    del cdf
    return w.to(torch.float32).contiguous(), S.view(n, n, n).to(torch.float32).contiguous()


def make_halos(cfg: BoxConfig, box: int = 0, device="cpu", w: torch.Tensor | None = None):
    """A halo catalogue for the box: (positions (n_halo, 3) FP32 in [0, L),
    masses (n_halo,) FP32), with host cells drawn with probability proportional
    to the density w (generated when not given), uniform positions inside the
    cell and masses from dN/dM ~ M^-1.9 on [m_lo, m_hi]."""
    n = cfg.n
    if w is None:
        w = make_density(n, config_seed(cfg.index, box), device=device,
                         dtype=torch.float64 if n <= 256 else torch.float32)
    gen = _gen(device, config_seed(cfg.index, box) + 11)
    cdf = torch.cumsum(w.reshape(-1).to(torch.float64), 0)
    u = torch.rand(cfg.n_halo, generator=gen, device=device, dtype=torch.float64) * cdf[-1].item()
    cell = torch.searchsorted(cdf, u).clamp_max(n * n * n - 1)
    del cdf, u
    cxyz = torch.stack([cell // (n * n), (cell // n) % n, cell % n], 1).to(torch.float64)
    off = torch.rand((cfg.n_halo, 3), generator=gen, device=device, dtype=torch.float64)
    pos = ((cxyz + off) * (cfg.box_len / n)).to(torch.float32)
    pos = torch.where(pos >= cfg.box_len, torch.zeros_like(pos), pos)   # float rounding at the top edge
    a, b = cfg.m_lo ** -0.9, cfg.m_hi ** -0.9
    um = torch.rand(cfg.n_halo, generator=gen, device=device, dtype=torch.float64)
    mass = ((a + um * (b - a)) ** (-1.0 / 0.9)).to(torch.float32)
    return pos.contiguous(), mass.contiguous()


def make_intensity(n: int, seed: int, device="cpu", ties: bool = True, negatives: bool = True) -> torch.Tensor:
    """A correlated FP32 intensity-like field for matching-only tests.

    Smooth (k^-3 GRF, exponentiated) with, when asked, planted exact ties
    (blocks of cells copied from other cells), signed zeros and negative values,
    which the ranking has to order exactly.
    """
    gen = _gen(device, seed)
    g = _grf(n, -3.0, gen, device, torch.float64 if n <= 256 else torch.float32)
    J = torch.exp(1.5 * g).to(torch.float32).reshape(-1)
    n3 = J.numel()
    if negatives:
        k = max(1, n3 // 50)
        idx = torch.randint(0, n3, (k,), generator=gen, device=device)
        J[idx] = -J[idx] * 1e-3
    if ties:
        k = max(2, n3 // 20)
        src = torch.randint(0, n3, (k,), generator=gen, device=device)
        dst = torch.randint(0, n3, (k,), generator=gen, device=device)
        J[dst] = J[src]
        z = torch.randint(0, n3, (max(2, n3 // 100),), generator=gen, device=device)
        half = z.numel() // 2
        J[z[:half]] = 0.0
        J[z[half:]] = -0.0
    return J.view(n, n, n).contiguous()


def make_weights_edge(n3: int, seed: int, kind: str, device="cpu") -> torch.Tensor:
    """Edge-case gas-mass weights: 'ones', 'wide' (exponent spread), 'subnormal'."""
    gen = _gen(device, seed)
    if kind == "ones":
        return torch.ones(n3, device=device, dtype=torch.float32)
    if kind == "wide":
        e = torch.randint(-40, 41, (n3,), generator=gen, device=device).to(torch.float64)
        m = 1.0 + torch.rand(n3, generator=gen, device=device, dtype=torch.float64)
        return (m * torch.pow(2.0, e)).to(torch.float32)
    if kind == "subnormal":
        w = (torch.rand(n3, generator=gen, device=device, dtype=torch.float64) + 0.5) * 1e-30
        w = w.to(torch.float32)
        k = max(2, n3 // 100)
        pick = torch.randint(0, n3, (k,), generator=gen, device=device)
        w[pick[: k // 2]] = torch.tensor(1e-40, dtype=torch.float32)     # FP32 subnormals
        w[pick[k // 2:]] = torch.tensor(1.4e-45, dtype=torch.float32)    # the smallest one
        return w
    raise ValueError(kind)


# ------------------------------------------------------------------------
# Mixed-size batches and a request stream (the batched and served workloads).

C4_SIZES = (64, 96, 128, 192, 256)
C3_LMFP = CONFIGS["c3"].l_mfp
C3_HISTORIES = CONFIGS["c3"].histories


def c4_boxes(count: int = 64, seed: int = 4, sizes=C4_SIZES):
    """``count`` boxes with N drawn uniformly from ``sizes``, L = 1.953125 N
    h^-1 Mpc, 1.3M (N/256)^3 halos on [1e10, 1e12], l_mfp ~ U[1, 20] and a
    history with z_mid ~ U[6, 10], Delta_z ~ U[2, 6], A_z ~ U[1.5, 4]."""
    g = torch.Generator().manual_seed(config_seed(seed, 0))
    out = []
    for b in range(count):
        n = sizes[int(torch.randint(0, len(sizes), (1,), generator=g))]
        u = torch.rand(4, generator=g, dtype=torch.float64).tolist()
        l = 1.0 + 19.0 * u[0]
        hist = (6.0 + 4.0 * u[1], 2.0 + 4.0 * u[2], 1.5 + 2.5 * u[3])
        out.append(BoxConfig(f"c4.{b}", n, 1.953125 * n, max(1000, int(1.3e6 * (n / 256) ** 3)), 1e10, 1e12,
                             l_mfp=(l,), histories=(hist,), index=100 + b))
    return out


def c5_requests(duration_s: float, rate_hz: float = 20.0, seed: int = 5, sizes=(128, 256, 512, 1024),
                weights=(0.4, 0.3, 0.2, 0.1)):
    """Poisson request stream: arrival times (exponential gaps at ``rate_hz``)
    over ``duration_s`` seconds, each with N drawn with ``weights`` and an
    l_mfp and history drawn from the swept sets of the 512^3 configuration."""
    g = torch.Generator().manual_seed(config_seed(seed, 0))
    cw = torch.tensor(weights, dtype=torch.float64).cumsum(0)
    t, reqs = 0.0, []
    while True:
        t += float(-math.log(1.0 - float(torch.rand(1, generator=g, dtype=torch.float64))) / rate_hz)
        if t >= duration_s:
            break
        u = float(torch.rand(1, generator=g, dtype=torch.float64)) * float(cw[-1])
        n = sizes[int((cw < u).sum())]
        li = int(torch.randint(0, len(C3_LMFP), (1,), generator=g))
        hi = int(torch.randint(0, len(C3_HISTORIES), (1,), generator=g))
        reqs.append((t, n, C3_LMFP[li], C3_HISTORIES[hi]))
    return reqs

"""Coefficients of the polynomial the radiation kernel uses for atan(x)/x.

The Fourier-space kernel of the radiation field is Khat(k) = atan(k l)/k =
l * g(k l) with g(x) = atan(x)/x, an even function with g(0) = 1.  On
0 <= x <= 1 the kernel evaluates g as P(x^2), P(t) = 1 + t Q(t) with Q of
degree DEG - 1; for x > 1 it uses atan(x) = pi/2 - atan(1/x), i.e.
g(x) = r (pi/2 - r g(r)) with r = 1/x, so P is only ever needed on [0, 1].

Q is a least-squares fit of (g(sqrt t) - 1)/t, weighted for relative error in
g, at Chebyshev nodes of [0, 1] (FP64).  The printed FP32 values are the ones
fft.hip holds (highest degree first, for Horner).  Run: python fit_atan.py
"""
from __future__ import annotations

import numpy as np

DEG = 9  # degree of P in t = x^2


def g(t: np.ndarray) -> np.ndarray:
    """atan(sqrt t)/sqrt t in FP64, 1 at t = 0."""
    t = np.asarray(t, dtype=np.float64)
    x = np.sqrt(t)
    out = np.ones_like(t)
    nz = x > 0
    out[nz] = np.arctan(x[nz]) / x[nz]
    return out


def fit(deg: int = DEG) -> np.ndarray:
    """P's coefficients c_0 = 1, c_1 .. c_deg (ascending), FP64."""
    m = 4 * deg + 1
    k = np.arange(m)
    t = 0.5 * (1.0 - np.cos(np.pi * (k + 0.5) / m))
    A = np.vander(t, deg, increasing=True) * t[:, None]     # t * t^j, j < deg
    w = 1.0 / g(t)
    q, *_ = np.linalg.lstsq(A * w[:, None], (g(t) - 1.0) * w, rcond=None)
    return np.concatenate([[1.0], q])


def coefficients_f32(deg: int = DEG) -> np.ndarray:
    return fit(deg).astype(np.float32)


def horner_f32(c32: np.ndarray, t: np.ndarray) -> np.ndarray:
    """P(t) evaluated in FP32 the way the kernel does (fused multiply-add per
    step, emulated as one FP64 multiply-add rounded to FP32, which is exact
    for the product of two FP32 values plus an FP32 value up to one rounding)."""
    t32 = np.asarray(t, dtype=np.float32)
    acc = np.full(t32.shape, c32[-1], dtype=np.float32)
    for a in c32[-2::-1]:
        acc = (acc.astype(np.float64) * t32.astype(np.float64) + np.float64(a)).astype(np.float32)
    return acc


if __name__ == "__main__":
    c = coefficients_f32()
    tt = np.linspace(0.0, 1.0, 200001)
    err = np.max(np.abs(horner_f32(c, tt).astype(np.float64) - g(tt)) / g(tt))
    print(f"// P(t) = atan(sqrt t)/sqrt t on [0, 1], degree {DEG}; FP32 Horner max relative error {err:.2e}")
    print("    " + ", ".join(f"{float(v):.9e}f" for v in c[::-1]))

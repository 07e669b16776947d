"""Pins for the oracle's radiation field (Sec. 3.4.1, Eq. intensity).

The oracle evaluates J = S * [exp(-r/l)/(4 pi r^2)] on the periodic grid as
IDFT[DFT(S) atan(k l)/k]/N^3.  Independent checks:
  * the closed-form kernel transform against numerical quadrature of the
    radial Fourier integral of exp(-r/l)/(4 pi r^2);
  * the naive DFT against numpy's FFT (a library routine);
  * the DFT route against a brute-force O(N^6) periodic convolution;
  * exact invariants: sum rule, linearity, translation covariance, realness;
  * a point source against the analytic periodic image sum (approximate: the
    sampled spectral kernel is truncated at the grid's Nyquist cube).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle


def _radial_transform(k, l_mfp):
    """(1/k) int_0^inf exp(-r/l) sin(kr)/r dr by adaptive quadrature over
    half-period pieces out to 60 attenuation lengths (e^-60 ~ 1e-26)."""
    f = lambda r: math.exp(-r / l_mfp) * (k * np.sinc(k * r / math.pi))
    step = min(math.pi / k, l_mfp)
    edges = np.arange(0.0, 60.0 * l_mfp + step, step)
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(f, a, b, epsabs=1e-15, epsrel=1e-13, limit=200)
        tot += v
    return tot / k


@pytest.mark.parametrize("l_mfp", [0.5, 3.0, 20.0])
@pytest.mark.parametrize("k", [1e-3, 0.05, 0.3, 2.0, 10.0])
def test_kernel_hat_vs_quadrature(k, l_mfp):
    """3D Fourier transform of a radial f(r): (4 pi / k) int r f(r) sin(kr) dr; with
    f = exp(-r/l)/(4 pi r^2) this is (1/k) int exp(-r/l) sin(kr)/r dr."""
    ref = _radial_transform(k, l_mfp)
    assert abs(oracle.kernel_hat(k, l_mfp) - ref) <= 1e-9 * max(1.0, abs(ref))


def test_kernel_hat_k0_limit():
    """Khat(0) = int exp(-r/l)/(4 pi r^2) d^3x = l_mfp, and continuity at small k."""
    for l in (0.5, 3.0, 50.0):
        assert oracle.kernel_hat(0.0, l) == l
        assert abs(oracle.kernel_hat(1e-7, l) - l) <= 1e-9 * l


def test_naive_dft_vs_numpy_fft():
    rng = np.random.default_rng(1)
    for n in (4, 6, 8, 12):
        x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
        assert np.allclose(oracle.dft3(x, -1), np.fft.fftn(x), rtol=0, atol=1e-11 * n ** 3)
        assert np.allclose(oracle.dft3(x, +1), np.fft.ifftn(x) * n ** 3, rtol=0, atol=1e-11 * n ** 3)


@pytest.mark.parametrize("n,L,l", [(8, 8.0, 1.5), (6, 12.0, 3.0), (8, 100.0 / 8, 0.4)])
def test_dft_route_vs_direct_convolution(n, L, l):
    """Brute force: J(x) = sum_x' S(x') g(x - x'), g = the kernel's periodic
    real-space form from a direct (non-separable) triple sum."""
    rng = np.random.default_rng(7)
    S = rng.random((n, n, n))
    J = oracle.radiation(S, L, l)
    Jd = oracle.direct_convolution(S, L, l)
    assert np.max(np.abs(J - Jd)) <= 1e-12 * np.max(np.abs(Jd))


def test_sum_rule_linearity_translation_realness():
    n, L, l = 16, 25.0, 3.0
    rng = np.random.default_rng(2)
    S1 = rng.random((n, n, n))
    S2 = rng.random((n, n, n)) ** 3
    J1, im = oracle.radiation(S1, L, l, return_imag=True)
    J2 = oracle.radiation(S2, L, l)
    # sum rule: the DC mode of J is Khat(0) = l_mfp times that of S
    assert math.isclose(J1.sum(), l * S1.sum(), rel_tol=1e-12)
    # linearity
    J12 = oracle.radiation(2.5 * S1 - 0.75 * S2, L, l)
    assert np.max(np.abs(J12 - (2.5 * J1 - 0.75 * J2))) <= 1e-12 * np.max(np.abs(J12))
    # periodic translation covariance
    sh = (3, -5, 7)
    Js = oracle.radiation(np.roll(S1, sh, axis=(0, 1, 2)), L, l)
    assert np.max(np.abs(Js - np.roll(J1, sh, axis=(0, 1, 2)))) <= 1e-12 * np.max(np.abs(J1))
    # real field in, real field out
    assert im <= 1e-12 * np.max(np.abs(J1))


def test_isotropy_and_monotone_profile():
    """A point source gives a field symmetric under axis permutations and
    reflections (the kernel depends on |k| only)."""
    n = 16
    S = np.zeros((n, n, n))
    S[0, 0, 0] = 1.0
    g = oracle.radiation(S, 16.0, 4.0)
    assert np.allclose(g, g.transpose(1, 0, 2), atol=1e-15)
    assert np.allclose(g, g.transpose(2, 1, 0), atol=1e-15)
    assert np.allclose(g, np.roll(g[::-1], 1, axis=0), atol=1e-15)
    prof = [g[r, r, r] for r in range(0, n // 2 + 1)]
    assert all(a > b for a, b in zip(prof[:-1], prof[1:]))


def _image_sum(dx, l, L, n_img=3):
    tot = 0.0
    for px in range(-n_img, n_img + 1):
        for py in range(-n_img, n_img + 1):
            for pz in range(-n_img, n_img + 1):
                r = math.sqrt((dx[0] + px * L) ** 2 + (dx[1] + py * L) ** 2 + (dx[2] + pz * L) ** 2)
                tot += math.exp(-r / l) / (4 * math.pi * r * r)
    return tot


def test_point_source_vs_periodic_image_sum():
    """Eq. (intensity) for a unit point source in a periodic box is the image sum
    of exp(-r/l)/(4 pi r^2).  The grid answer with l_c = 1 is J per unit mass.
    The sampled spectral kernel is cut off at the Nyquist cube, whose ringing
    runs along the grid axes; off the axes the two agree closely: along the
    body diagonal to < 2e-4 from r = 3 cells on, improving with r, and along a
    face diagonal to ~1%."""
    n, L, l = 32, 32.0, 8.0          # l_c = 1
    S = np.zeros((n, n, n))
    S[0, 0, 0] = 1.0
    g = oracle.radiation(S, L, l)     # per unit cell volume (l_c = 1)
    body = {r: abs(g[r, r, r] / _image_sum((r, r, r), l, L) - 1) for r in (3, 4, 6, 8, 12)}
    assert body[3] < 2e-4 and body[8] < 3e-5 and body[12] < 1e-5
    assert body[12] < body[8] < body[4] < body[3]
    face = max(abs(g[r, r, 0] / _image_sum((r, r, 0), l, L) - 1) for r in (3, 4, 6, 8, 12))
    assert face < 0.015
    # the 4 pi and the attenuation length are both pinned: a factor 4 pi off or
    # l -> l/2 would miss by far more than these bounds
    far = (6, 6, 6)
    assert abs(g[far] / _image_sum(far, l / 2, L) - 1) > 0.3
    assert abs(g[far] / (4 * math.pi * _image_sum(far, l, L)) - 1) > 0.3


def test_negative_values_from_spectral_ringing():
    """Reading R3: the sampled kernel's real-space form rings, so J of a
    non-negative source can be slightly negative far from sources."""
    n = 32
    S = np.zeros((n, n, n))
    S[0, 0, 0] = 1.0
    g = oracle.radiation(S, 50.0, 3.0)           # l_c = 1.5625, l_mfp ~ 1.9 cells
    assert g.min() < 0 and abs(g.min()) < 1e-2 * g.max()
    assert 0.01 < np.mean(g < 0) < 0.6
    assert math.isclose(g.sum(), 3.0, rel_tol=1e-12)


@pytest.mark.parametrize("n", [4, 6, 8, 12, 16])
def test_dft_coeff_matches_numpy_fft(n):
    """oracle_dft_coeff_f32 (one DFT coefficient of an FP32 field, the checker
    of full-size transforms) against numpy's FFT at every mode of small grids."""
    rng = np.random.default_rng(1000 + n)
    f = rng.standard_normal((n, n, n)).astype(np.float32)
    ref = np.fft.fftn(f.astype(np.float64))
    scale = np.sqrt(np.sum(np.abs(ref) ** 2) / ref.size)
    worst = 0.0
    for m in np.ndindex(n, n, n):
        got = oracle.dft_coeff(f, m)
        worst = max(worst, abs(got - ref[m]) / scale)
    assert worst <= 1e-12, worst

"""Pins of the oracle's two-point statistics (Sec. 2.3, Eqs. deltaz, Pk, Dk,
bias, rcc; readings D1 field normalisations, D2 shell averages) against
numpy's FFT with numpy binning, Parseval's theorem, a plane wave, exact
bias/correlation cases and the white-noise expectation."""
import numpy as np
import pytest

import oracle

def _shells_numpy(n, n_bins):
    m = np.fft.fftfreq(n, 1.0 / n)          # signed integer frequencies
    s2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    sh = np.floor(np.sqrt(s2) + 0.5).astype(np.int64)   # (i + 1/2)^2 is never an integer
    return s2, sh


def _numpy_spectra(a, b, L, n_bins):
    n = a.shape[0]
    A, B = np.fft.fftn(a), np.fft.fftn(b)
    s2, sh = _shells_numpy(n, n_bins)
    keep = sh < n_bins
    cnt = np.bincount(sh[keep], minlength=n_bins).astype(float)
    vol = L ** 3 / float(n) ** 6
    paa = np.bincount(sh[keep], weights=np.abs(A[keep]) ** 2, minlength=n_bins)
    pbb = np.bincount(sh[keep], weights=np.abs(B[keep]) ** 2, minlength=n_bins)
    pab = np.bincount(sh[keep], weights=(A[keep] * np.conj(B[keep])).real, minlength=n_bins)
    kk = np.bincount(sh[keep], weights=np.sqrt(s2[keep]), minlength=n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        return cnt, 2 * np.pi / L * kk / cnt, vol * paa / cnt, vol * pbb / cnt, vol * pab / cnt


@pytest.mark.parametrize("n", [6, 8, 12, 16])
def test_matches_numpy_fft_and_binning(n):
    rng = np.random.default_rng(n)
    a = rng.normal(size=(n, n, n))
    b = 0.5 * a + rng.normal(size=(n, n, n))
    L, nb = 3.0 * n, n
    s = oracle.spectra(a, b, L, nb)
    cnt, k, paa, pbb, pab = _numpy_spectra(a, b, L, nb)
    assert np.array_equal(s["modes"], cnt)
    ok = cnt > 0
    for got, ref in ((s["k"], k), (s["p_aa"], paa), (s["p_bb"], pbb), (s["p_ab"], pab)):
        assert np.allclose(got[ok], ref[ok], rtol=1e-10, atol=1e-12 * np.max(np.abs(ref[ok])))


def test_parseval():
    n, L = 16, 20.0
    rng = np.random.default_rng(1)
    a = rng.normal(size=(n, n, n)) + 0.3
    nb = int(np.ceil(np.sqrt(3) * n / 2)) + 2          # every mode in some shell
    s = oracle.spectra(a, None, L, nb)
    assert s["modes"].sum() == n ** 3
    total = np.sum(s["modes"] * s["p_aa"]) * n ** 6 / L ** 3
    assert total == pytest.approx(n ** 3 * np.sum(a ** 2), rel=1e-12)


def test_plane_wave_single_shell():
    n, L = 16, 10.0
    m0 = (3, 4, 0)                                      # |m| = 5
    x = np.indices((n, n, n))
    a = np.cos(2 * np.pi * (m0[0] * x[0] + m0[1] * x[1] + m0[2] * x[2]) / n)
    s = oracle.spectra(a, None, L, 10)
    expect = L ** 3 / n ** 6 * (2 * (n ** 3 / 2.0) ** 2) / s["modes"][5]
    assert s["p_aa"][5] == pytest.approx(expect, rel=1e-12)
    others = np.delete(s["p_aa"], 5)
    assert np.max(np.abs(others)) <= 1e-20 * expect


def test_bias_and_correlation_exact_cases():
    n, L = 12, 12.0
    rng = np.random.default_rng(2)
    a = rng.normal(size=(n, n, n))
    nb = 7
    two = oracle.spectra(2.0 * a, a, L, nb)
    ok = two["modes"] > 0
    assert np.allclose(two["bias"][ok][1:], 2.0, rtol=1e-12)
    assert np.allclose(two["r"][ok][1:], 1.0, rtol=1e-12)
    neg = oracle.spectra(-a, a, L, nb)
    assert np.allclose(neg["r"][ok][1:], -1.0, rtol=1e-12)
    # an independent field: correlation well inside (-1, 1) in every shell with many modes
    ind = oracle.spectra(a, rng.normal(size=(n, n, n)), L, nb)
    assert np.all(np.abs(ind["r"][ind["modes"] > 200]) < 0.3)


def test_field_normalisations():
    n, L = 12, 30.0
    rng = np.random.default_rng(3)
    f = np.exp(0.5 * rng.normal(size=(n, n, n)))
    od1 = oracle.spectra(f, None, L, 8, kind_a=oracle.FIELD_OVERDENSITY)
    od2 = oracle.spectra(7.5 * f, None, L, 8, kind_a=oracle.FIELD_OVERDENSITY)
    assert np.allclose(od1["p_aa"], od2["p_aa"], rtol=1e-12)
    assert od1["p_aa"][0] <= 1e-25                     # the mean is removed
    raw = oracle.spectra(f / f.mean() - 1.0, None, L, 8)
    assert np.allclose(od1["p_aa"][1:], raw["p_aa"][1:], rtol=1e-10)
    z = 8.0 + rng.normal(size=(n, n, n))
    dz = oracle.spectra(z, None, L, 8, kind_a=oracle.FIELD_REDSHIFT)
    zbar = z.mean()
    raw_z = oracle.spectra((z - zbar) / (1.0 + zbar), None, L, 8)
    assert np.allclose(dz["p_aa"][1:], raw_z["p_aa"][1:], rtol=1e-10)
    assert dz["p_aa"][0] <= 1e-20 * dz["p_aa"][1]      # mean removed: only rounding left


def test_white_noise_is_flat():
    n, L, sigma = 32, 64.0, 1.7
    rng = np.random.default_rng(4)
    a = sigma * rng.normal(size=(n, n, n))
    s = oracle.spectra(a, None, L, 16)
    expect = sigma ** 2 * (L / n) ** 3                   # variance times the cell volume
    for i in range(4, 16):
        # each shell averages many independent |A_m|^2 (pairs of conjugate modes)
        tol = 5.0 / np.sqrt(s["modes"][i] / 2.0)
        assert abs(s["p_aa"][i] / expect - 1.0) <= tol, i

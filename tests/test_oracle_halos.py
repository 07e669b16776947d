"""Pins of the oracle's halo source construction (Sec. 3.2.1, Eqs. interlace,
Wofk; readings A1, A2):

  * the CIC deposit against the input generator's independent torch CIC, the
    NGP deposit against numpy binning, the TSC weights against their closed
    form, mass conservation for every scheme;
  * the sum rule of the radiation field and translation covariance;
  * the deconvolved (and interlaced) spectrum of a single halo against the
    ideal point source e^{-i k.(x_h - x_0)} at low k, with interlacing reducing
    the aliasing error at higher k.
"""
import numpy as np
import pytest
import torch

import oracle
from inputs.synth import _cic_deposit


def _halos(n_halo, L, seed):
    rng = np.random.default_rng(seed)
    pos = (rng.random((n_halo, 3)) * L).astype(np.float32)
    mass = (10 ** rng.uniform(0, 2, n_halo)).astype(np.float32)
    return pos, mass


def test_cic_matches_independent_deposit():
    n, L = 16, 40.0
    pos, mass = _halos(300, L, 1)
    mesh = oracle.deposit(n, L, pos, mass, oracle.CIC)
    ref = _cic_deposit(n, torch.from_numpy(pos.astype(np.float64) * (n / L)),
                       torch.from_numpy(mass.astype(np.float64)), torch.float64).numpy()
    assert np.allclose(mesh, ref, rtol=1e-12, atol=1e-12 * mass.max())


def test_ngp_matches_binning():
    n, L = 12, 30.0
    pos, mass = _halos(500, L, 2)
    mesh = oracle.deposit(n, L, pos, mass, oracle.NGP)
    idx = np.floor(pos.astype(np.float64) * (n / L)).astype(np.int64) % n
    flat = (idx[:, 0] * n + idx[:, 1]) * n + idx[:, 2]
    ref = np.bincount(flat, weights=mass.astype(np.float64), minlength=n ** 3).reshape(n, n, n)
    assert np.allclose(mesh, ref, rtol=1e-14, atol=0)


def test_tsc_weights_closed_form():
    n, L = 8, 8.0
    # a halo on a node centre: weights 1/8, 3/4, 1/8 per axis
    mesh = oracle.deposit(n, L, np.array([[3.5, 3.5, 3.5]], np.float32), np.array([1.0], np.float32), oracle.TSC)
    w1 = np.array([0.125, 0.75, 0.125])
    assert np.allclose(mesh[2:5, 2:5, 2:5], np.einsum("i,j,k->ijk", w1, w1, w1), rtol=1e-15)
    # a halo on a cell face (u = -1/2): weights 1/2, 1/2, 0
    mesh = oracle.deposit(n, L, np.array([[3.0, 3.5, 3.5]], np.float32), np.array([1.0], np.float32), oracle.TSC)
    assert mesh[2, 3, 3] == pytest.approx(0.5 * 0.75 * 0.75) and mesh[3, 3, 3] == pytest.approx(0.5 * 0.75 * 0.75)
    for p in (oracle.NGP, oracle.CIC, oracle.TSC):
        pos, mass = _halos(200, L, 3 + p)
        for shift in (0.0, 0.5):
            assert oracle.deposit(n, L, pos, mass, p, shift).sum() == pytest.approx(
                mass.astype(np.float64).sum(), rel=1e-13)


@pytest.mark.parametrize("p,inter", [(1, False), (2, False), (2, True), (3, True)])
def test_sum_rule_and_translation(p, inter):
    n, L, l = 16, 32.0, 3.0
    pos, mass = _halos(40, L, 10 + p)
    J = oracle.radiation_from_halos(n, L, pos, mass, p, inter, l)
    assert J.sum() == pytest.approx(l * mass.astype(np.float64).sum(), rel=1e-11)
    shift = np.array([3, 5, 2])
    pos2 = ((pos.astype(np.float64) + shift * (L / n)) % L).astype(np.float32)
    J2 = oracle.radiation_from_halos(n, L, pos2, mass, p, inter, l)
    # shifted float32 positions round differently in their last bits (~1e-7 of
    # a cell), which bounds the difference
    assert np.allclose(np.roll(J, tuple(shift), axis=(0, 1, 2)), J2, rtol=1e-5, atol=1e-6 * np.abs(J).max())


def test_deconvolved_spectrum_of_a_point_source():
    n, L, l = 32, 32.0, 3.0
    x = np.array([[10.3, 17.71, 5.45]], np.float32)
    m = np.array([1.0], np.float32)
    s = np.fft.fftfreq(n, 1.0 / n)
    S = np.meshgrid(s, s, s, indexing="ij")
    k = 2 * np.pi / L * np.sqrt(S[0] ** 2 + S[1] ** 2 + S[2] ** 2)
    K = np.where(k > 0, np.arctan(k * l) / np.where(k > 0, k, 1.0), l)
    xs = x[0].astype(np.float64) - 0.5 * L / n          # relative to the first node (cell centre 0)
    ideal = np.exp(-2j * np.pi / L * (S[0] * xs[0] + S[1] * xs[1] + S[2] * xs[2]))
    err = {}
    for inter in (False, True):
        J = oracle.radiation_from_halos(n, L, x, m, oracle.CIC, inter, l)
        X = np.fft.fftn(J) / K
        err[inter] = {mm: abs(X[mm] - ideal[mm]) for mm in [(1, 0, 0), (0, 2, 1), (3, 1, 2), (8, 0, 0), (4, 4, 4)]}
    for mm in [(1, 0, 0), (0, 2, 1), (3, 1, 2)]:
        assert err[True][mm] <= 3e-3, mm
    # the half-cell diagonal shift cancels the aliases displaced by an odd
    # number of periods, the leading ones for these modes
    for mm in [(3, 1, 2), (8, 0, 0), (4, 4, 4)]:
        assert err[True][mm] < 0.5 * err[False][mm], mm

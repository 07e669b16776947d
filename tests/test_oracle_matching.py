"""Pins for the oracle's abundance matching (Sec. 3.4.2).

Independent checks: numpy's lexsort for the rank order, Python's exact
rational arithmetic (fractions) for the cumulative mass and its rounding, the
closed form for unit weights, and the invariants the paper states: matching
does not depend on the field's normalisation (Secs. 3.4, 5.1), cells ranked
at or before n are ionized, and the ionized mass fraction equals x_i(z).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

import inputs
import oracle

HIST = oracle.History.from_params(8.0, 4.0, 3.0)


def _lexsort_rank(J):
    flat = np.asarray(J).reshape(-1)
    idx = np.arange(flat.size)
    return np.lexsort((idx, -flat.astype(np.float64))).astype(np.uint32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rank_vs_lexsort_with_ties_zeros_negatives(seed):
    J = inputs.make_intensity(16, 100 + seed).numpy()
    assert (J == 0).sum() > 0 and (J < 0).sum() > 0
    assert np.unique(J).size < J.size                      # planted ties
    assert np.array_equal(oracle.rank(J), _lexsort_rank(J))


def test_rank_signed_zero_and_adversarial():
    J = np.array([0.0, -0.0, 1.0, -1.0, 0.0, np.float32(1e-45), -np.float32(1e-45),
                  3.4e38, -3.4e38, np.inf, -np.inf, 1.0, -0.0], dtype=np.float32)
    perm = oracle.rank(J)
    assert list(perm) == [9, 7, 2, 11, 5, 0, 1, 4, 12, 6, 3, 8, 10]
    for J2 in (np.zeros(37, np.float32), np.arange(50, dtype=np.float32),
               np.arange(50, dtype=np.float32)[::-1].copy()):
        assert np.array_equal(oracle.rank(J2), _lexsort_rank(J2))


def test_rank_nan_rejected():
    J = np.ones(10, dtype=np.float32)
    J[4] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.rank(J)
    assert e.value.code == oracle.E_DATA


def _exact_F(perm, w):
    fr = [Fraction(float(x)) for x in w]
    tot = sum(fr)
    out, c = [], Fraction(0)
    for p in perm:
        c += fr[p]
        out.append(float(c) / float(tot))     # int/Fraction -> float is correctly rounded
    return np.array(out)


@pytest.mark.parametrize("kind", ["lognormal", "wide", "subnormal", "ones"])
def test_mass_fraction_exact_vs_fractions(kind):
    n3 = 4096
    if kind == "lognormal":
        w = inputs.make_density(16, 11).numpy().astype(np.float32).reshape(-1)
    else:
        w = inputs.make_weights_edge(n3, 12, kind).numpy()
    rng = np.random.default_rng(5)
    perm = rng.permutation(w.size).astype(np.uint32)
    F = oracle.mass_fraction(perm, w)
    assert np.array_equal(F, _exact_F(perm, w))
    assert F[-1] == 1.0 and np.all(np.diff(F) >= 0)


def test_unit_weights_closed_form():
    """w = 1: F_n = n/N exactly (volume weighting, Sec. 3.1), so z_n is the
    closed-form inverse evaluated at n/N."""
    n3 = 4096
    w = np.ones(n3, dtype=np.float32)
    perm = np.arange(n3, dtype=np.uint32)
    F = oracle.mass_fraction(perm, w)
    assert np.array_equal(F, np.arange(1, n3 + 1) / n3)
    J = np.linspace(5, -5, n3).astype(np.float32)
    z32, z64 = oracle.zre(J, w, HIST, mode=oracle.EXACT)
    ref = HIST.a + HIST.b * (-np.log(np.arange(1, n3 + 1) / n3)) ** (1 / HIST.c)
    assert np.allclose(z64, ref, rtol=1e-13, atol=1e-13)


def test_u128_rounding_to_nearest_even():
    cases = [(1 << 53) + 1, (1 << 53) + 3, (1 << 54) + 2, (1 << 54) + 6, (1 << 64) - 1,
             (1 << 100) + (1 << 47), (1 << 100) + (1 << 47) + 1, (1 << 127) - 1,
             (1 << 126) + (1 << 73) + (1 << 72), 12345678901234567890123456789]
    for v in cases:
        assert oracle.u128_to_double(v) == float(v), hex(v)


def test_weight_errors():
    J = np.arange(16, dtype=np.float32)
    for bad in (0.0, -1.0, np.inf, np.nan):
        w = np.ones(16, dtype=np.float32)
        w[3] = bad
        with pytest.raises(oracle.OracleError) as e:
            oracle.zre(J, w, HIST)
        assert e.value.code == oracle.E_DATA
    w = np.ones(16, dtype=np.float32)
    w[0], w[1] = np.float32(1e-40), np.float32(3e38)     # > 103-bit shift
    with pytest.raises(oracle.OracleError) as e:
        oracle.zre(J, w, HIST)
    assert e.value.code == oracle.E_RANGE


def _box(n=24, seed=3):
    w = inputs.make_density(n, seed).numpy().astype(np.float32)
    J = inputs.make_intensity(n, seed + 1).numpy()
    return J, w


def test_ionized_mass_fraction_matches_history():
    """Sec. 3.4.2: the mass with z_re > z equals x_i(z) to within one cell's mass
    (the last cell crossing z), at every z."""
    J, w = _box()
    z32, z64 = oracle.zre(J, w, HIST, mode=oracle.EXACT)
    wf = w.reshape(-1).astype(np.float64)
    order = np.argsort(-z64.reshape(-1), kind="stable")
    tot = wf.sum()
    for z in np.linspace(HIST.a - 0.5, 16.0, 200):
        frac = wf[z64.reshape(-1) > z].sum() / tot
        xi = oracle.lib().oracle_weibull_x(z, HIST.a, HIST.b, HIST.c)
        assert abs(frac - xi) <= wf.max() / tot + 1e-12, z
    assert order.size == wf.size


def test_monotone_and_range():
    """z_re is non-increasing along the rank order (higher intensity ionizes
    earlier), lies in [a_w, z_top], and the last-ranked cell gets a_w."""
    J, w = _box()
    for mode in (oracle.EXACT, oracle.CONTRACT):
        z32, z64, perm = oracle.zre(J, w, HIST, mode=mode, want_perm=True)
        zs = z64.reshape(-1)[perm]
        assert np.all(np.diff(zs) <= 0)
        assert zs[-1] == HIST.a
        assert np.all(zs >= HIST.a) and np.all(zs <= HIST.z_top)


def test_normalisation_and_monotone_map_invariance():
    """Matching ignores the normalisation of the correlated field (Sec. 3.4.1) and
    depends only on rank order: 2^k J, or any strictly increasing map of J, gives
    bit-identical z_re."""
    J, w = _box()
    base, _ = oracle.zre(J, w, HIST)
    # exact power-of-two scalings in FP32, and the cube in FP64 (strictly
    # increasing, and distinct FP32 inputs stay distinct)
    for J2 in (J * np.float32(8.0), J * np.float32(2.0 ** -20), J.astype(np.float64) ** 3):
        assert np.array_equal(oracle.rank(J2), oracle.rank(J))
        z2, _ = oracle.zre(J2, w, HIST)
        assert np.array_equal(z2, base)


def test_cells_one_by_one_equal_full_match():
    J, w = _box(16, 9)
    z_full, _ = oracle.zre(J, w, HIST)
    rng = np.random.default_rng(0)
    cells = np.concatenate([rng.integers(0, J.size, 20), [0, J.size - 1]])
    zc, F = oracle.zre_cells(J, w, cells, HIST)
    assert np.array_equal(zc, z_full.reshape(-1)[cells])


def test_end_to_end_small_box():
    """64^3 configuration end to end in FP64: radiation then matching."""
    cfg = inputs.CONFIGS["c1"]
    w, S = inputs.make_box(cfg)
    J, im = oracle.radiation(S.numpy().astype(np.float64), cfg.box_len, cfg.l_mfp[0], return_imag=True)
    assert im <= 1e-12 * np.abs(J).max()
    assert math.isclose(J.sum(), cfg.l_mfp[0] * float(S.double().sum()), rel_tol=1e-10)
    z32, z64 = oracle.zre(J, w.numpy(), HIST, mode=oracle.EXACT)
    wf = w.numpy().reshape(-1).astype(np.float64)
    frac = wf[z64.reshape(-1) > 8.0].sum() / wf.sum()
    assert abs(frac - 0.5) <= wf.max() / wf.sum() + 1e-12
    # cells with more source mass nearby reionize earlier on average
    dens_rank_corr = np.corrcoef(z64.reshape(-1), np.log(J.reshape(-1) - J.min() + 1e-30))[0, 1]
    assert dens_rank_corr > 0.5
    assert torch.is_tensor(w)

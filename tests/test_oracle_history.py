"""Pins for the oracle's reionization history (Sec. 3.1, Appendix A).

Each check is tied to something other than the oracle itself: the worked
example printed in Table 1, the closed forms of Eqs. (duration), (asymmetry)
and (weibull), and a high-precision decimal evaluation of the table entries.
"""
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_weibull.txt")


def _table1():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, *vals = line.split()
        rows.append((name, *map(float, vals)))
    return rows


@pytest.mark.parametrize("row", _table1(), ids=lambda r: r[0])
def test_table1_worked_example(row):
    """Table 1: (z_mid, Delta_z, A_z) -> (a_w, b_w, c_w) to the printed precision.

    The printed inputs are rounded to 0.01, so the printed outputs must be
    reachable from some input inside the +-0.005 rounding box.
    """
    name, zm, dz, az, a_p, b_p, c_p = row
    a, b, c = oracle.weibull_fit(zm, dz, az)
    assert abs(a - a_p) <= 0.0101 and abs(b - b_p) <= 0.0101 and abs(c - c_p) <= 0.0051
    lo = np.array([np.inf] * 3)
    hi = -lo
    for dzm in (-0.005, 0.0, 0.005):
        for ddz in (-0.005, 0.0, 0.005):
            for daz in (-0.005, 0.0, 0.005):
                v = np.array(oracle.weibull_fit(zm + dzm, dz + ddz, az + daz))
                lo = np.minimum(lo, v)
                hi = np.maximum(hi, v)
    for p, l, h in zip((a_p, b_p, c_p), lo, hi):
        # the printed value's rounding interval overlaps the image of the input box
        assert l - 0.005 <= p <= h + 0.005


def test_table1_sim1_sim2_exact_digits():
    """Sims 1 and 2 reproduce all printed digits without input perturbation."""
    for name, zm, dz, az, a_p, b_p, c_p in _table1()[1:]:
        a, b, c = oracle.weibull_fit(zm, dz, az)
        assert (round(a, 2), round(b, 2), round(c, 2)) == (a_p, b_p, c_p), name


@pytest.mark.parametrize("hist", [(8.0, 4.0, 3.0), (7.95, 4.68, 2.90), (6.0, 2.0, 1.5),
                                  (10.0, 6.0, 4.0), (9.0, 3.0, 1.0), (8.0, 4.0, 12.0)])
def test_history_points_closed_form(hist):
    """Eqs. (duration), (asymmetry): the points give back Delta_z and A_z, and the
    fitted Weibull passes through (z_ear, 0.05), (z_mid, 0.5), (z_lat, 0.95)."""
    zm, dz, az = hist
    ze, zl = oracle.history_points(zm, dz, az)
    assert ze > zm > zl
    assert math.isclose(ze - zl, dz, rel_tol=0, abs_tol=1e-13)
    assert math.isclose((ze - zm) / (zm - zl), az, rel_tol=1e-12)
    a, b, c = oracle.weibull_fit(zm, dz, az)
    for z, x in ((ze, 0.05), (zm, 0.5), (zl, 0.95)):
        assert abs(oracle.lib().oracle_weibull_x(z, a, b, c) - x) <= 1e-12
        assert abs(oracle.lib().oracle_weibull_z(x, a, b, c) - z) <= 1e-11


def test_custom_ionization_points():
    """Users may pick other points (Sec. 3.1.1), e.g. quartiles (0.25, 0.5, 0.75)."""
    zm, dz, az = 8.0, 2.0, 1.8
    a, b, c = oracle.weibull_fit(zm, dz, az, 0.25, 0.5, 0.75)
    ze, zl = oracle.history_points(zm, dz, az)
    for z, x in ((ze, 0.25), (zm, 0.5), (zl, 0.75)):
        assert abs(oracle.lib().oracle_weibull_x(z, a, b, c) - x) <= 1e-12


def test_weibull_shape_properties():
    """Eq. (weibull): x = 1 at and below a_w (the max() term), monotone decreasing
    above, and the inverse is the closed form a_w + b_w |ln x|^(1/c_w)."""
    a, b, c = oracle.weibull_fit(8.0, 4.0, 3.0)
    L = oracle.lib()
    assert L.oracle_weibull_x(a, a, b, c) == 1.0
    assert L.oracle_weibull_x(a - 1.0, a, b, c) == 1.0
    zs = np.linspace(a + 1e-3, a + 30, 500)
    xs = np.array([L.oracle_weibull_x(z, a, b, c) for z in zs])
    assert np.all(np.diff(xs) < 0)
    for z, x in zip(zs[::50], xs[::50]):
        assert math.isclose(a + b * abs(math.log(x)) ** (1 / c), z, rel_tol=1e-12)


def test_trends_with_parameters():
    """Sec. 3.1.2: b_w grows with Delta_z; c_w is inversely related to A_z."""
    _, b1, _ = oracle.weibull_fit(8.0, 3.0, 3.0)
    _, b2, _ = oracle.weibull_fit(8.0, 5.0, 3.0)
    assert b2 > b1
    cs = [oracle.weibull_fit(8.0, 4.0, az)[2] for az in (1.5, 2.0, 3.0, 4.0, 8.0)]
    assert all(x > y for x, y in zip(cs, cs[1:]))


@pytest.mark.parametrize("bad", [(8.0, 4.0, 0.5), (8.0, 4.0, 16.0), (8.0, 0.0, 3.0),
                                 (8.0, -1.0, 3.0), (8.0, 4.0, -2.0), (1.0, 6.0, 3.0)])
def test_history_rejected(bad):
    """No positive (a_w, b_w, c_w) (Sec. 3.1.2 requires all positive), A_z beyond
    the paper's stated range, or a non-positive duration -> error."""
    with pytest.raises(oracle.OracleError):
        oracle.weibull_fit(*bad)


def test_root_exists_above_asymptote():
    """As c_w -> infinity the asymmetry tends to
    ln(L_e/L_m)/ln(L_m/L_l) (L = |ln x|); just above it a root exists."""
    Le, Lm, Ll = abs(math.log(0.05)), abs(math.log(0.5)), abs(math.log(0.95))
    amin = math.log(Le / Lm) / math.log(Lm / Ll)
    assert 0.56 < amin < 0.57
    # a_w > 0 also has to hold: pick a high z_mid so the late end stays positive
    a, b, c = oracle.weibull_fit(40.0, 4.0, amin * 1.07)
    assert c > 20 and a > 0
    with pytest.raises(oracle.OracleError):
        oracle.weibull_fit(40.0, 4.0, amin * 0.99)


def _decimal_x(z_j: float, a: float, b: float, c: float) -> float:
    getcontext().prec = 50
    u = (Decimal(z_j) - Decimal(a)) / Decimal(b)
    if u <= 0:
        return 1.0
    return float((-(u ** Decimal(c))).exp())


@pytest.mark.parametrize("hist", [(8.0, 4.0, 3.0), (7.83, 6.54, 2.33), (10.0, 6.0, 4.0)])
def test_table_against_decimal(hist):
    """Contract-table entries X_j = x_i(z_j): monotone, X_0 = 1, covering
    F >= 2^-64, each within the FP64 error bound of a 50-digit decimal evaluation
    of the same node: 4 ulp times the condition number 1 + c_w |ln X_j| of
    exp(-u^c_w) with respect to u."""
    H = oracle.History.from_params(*hist)
    X = H.X
    assert X[0] == 1.0
    assert np.all(np.diff(X) <= 0)
    assert X[-1] <= 2.0 ** -64 * (1 + 1e-9)
    assert H.T <= 2 ** 22 and H.h == 2.0 ** round(math.log2(H.h))
    rng = np.random.default_rng(3)
    for j in np.concatenate([[0, 1, 2, H.T - 1, H.T], rng.integers(0, H.T, 60)]):
        z_j = H.a + float(j) * H.h
        ref = _decimal_x(z_j, H.a, H.b, H.c)
        cond = 1.0 + H.c * abs(math.log(ref))
        assert abs(X[j] - ref) <= 4 * cond * np.spacing(ref), j


def test_contract_vs_exact_inversion_within_h():
    """Table interpolation differs from the closed-form inverse by at most h, hits
    the nodes exactly, maps F = 1 to a_w (reading Z5) and clamps at z_top."""
    for hist in [(8.0, 4.0, 3.0), (10.0, 6.0, 4.0), (6.0, 2.0, 1.5)]:
        H = oracle.History.from_params(*hist)
        rng = np.random.default_rng(0)
        F = np.concatenate([10.0 ** rng.uniform(-19, 0, 2000), [1.0, 0.5, 2.0 ** -64]])
        zc = oracle.invert(F, H, oracle.CONTRACT)
        ze = oracle.invert(F, H, oracle.EXACT)
        assert np.max(np.abs(zc - ze)) <= H.h
        assert zc[-3] == H.a and ze[-3] == H.a
        assert np.all(zc <= H.z_top) and np.all(ze <= H.z_top)
        assert np.all(np.diff(zc[np.argsort(F)]) <= 0)        # monotone in F
        js = rng.integers(1, H.T - 1, 50)
        zn = oracle.invert(H.X[js], H, oracle.CONTRACT)
        assert np.array_equal(zn, H.a + js.astype(np.float64) * H.h)

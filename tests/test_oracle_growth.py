"""Pins of the oracle's growth-rescaled matching (Sec. 3.4.2 with
delta_m(z) = D(z)/D(z_mid) delta_m; readings G1, G2):

  * D(z) against a direct quadrature of the growing-mode integral of a flat
    matter + Lambda universe (an independent formula), its matter-dominated
    limit D = a and the matter-only case;
  * the node tables against that quadrature;
  * the matched z_re against a brute-force root of the continuous equation
    (scipy brentq on exact D and exact x_i) on a small grid, within the node
    spacing h;
  * with G = 1 it reduces to the plain matching up to rounding.
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import inputs
import oracle


def _growth_quad(z, om):
    """D(a) = (5 om / 2) E(a) int_0^a da' / (a' E(a'))^3, E = sqrt(om a^-3 + 1 - om)."""
    a = 1.0 / (1.0 + z)
    E = lambda x: math.sqrt(om / x ** 3 + 1.0 - om)
    val, _ = integrate.quad(lambda x: 1.0 / (x * E(x)) ** 3, 0.0, a, epsabs=0, epsrel=1e-13, limit=200)
    return 2.5 * om * E(a) * val


@pytest.mark.parametrize("z", [0.0, 0.3, 1.0, 3.0, 6.0, 8.0, 12.0, 30.0])
@pytest.mark.parametrize("om", [0.3, 0.5, 0.1])
def test_growth_matches_quadrature(z, om):
    assert oracle.growth(z, om) == pytest.approx(_growth_quad(z, om), rel=1e-10)


def test_growth_limits():
    for z in (0.0, 2.0, 9.0):
        assert oracle.growth(z, 1.0) == pytest.approx(1.0 / (1.0 + z), rel=1e-15)   # matter only: D = a
    assert oracle.growth(1000.0, 0.3) == pytest.approx(1.0 / 1001.0, rel=1e-8)     # matter dominated early
    # growth suppression today for the paper's cosmology
    assert 0.77 < oracle.growth(0.0, 0.3) < 0.79


def test_growth_table_nodes():
    H = oracle.History.from_params(8.0, 4.0, 3.0)
    G = oracle.growth_table(H, 8.0)
    assert G.size == H.T + 1
    d8 = _growth_quad(8.0, 0.3)
    for j in (0, 1, H.T // 3, H.T // 2, H.T):
        z = H.a + j * H.h
        assert G[j] == pytest.approx(_growth_quad(z, 0.3) / d8, rel=1e-10)
    assert np.all(np.diff(G) < 0)          # later nodes are at higher z: less growth


def _masses(J, w):
    perm = oracle.rank(J)
    wp = w.reshape(-1)[perm].astype(np.float64)
    return perm, np.cumsum(wp), wp.sum()


def test_brute_force_continuous_root():
    n = 8
    J = inputs.make_intensity(n, 601, ties=False, negatives=False).numpy()
    w = inputs.make_density(n, 602).numpy().astype(np.float32)
    H = oracle.History.from_params(8.0, 4.0, 3.0)
    G = oracle.growth_table(H, 8.0)
    z32, z64 = oracle.zre_growth(J, w, H, G)
    perm, C, Ctot = _masses(J, w)
    N = J.size
    d_mid = _growth_quad(8.0, 0.3)
    worst = 0.0
    for k in range(N):
        cnt = k + 1

        def f(z):
            g = _growth_quad(z, 0.3) / d_mid
            m = cnt * (1 - g) + g * C[k]
            M = N * (1 - g) + g * Ctot
            return m / M - math.exp(-(((z - H.a) / H.b) ** H.c))

        lo, hi = H.a, H.z_top
        if f(lo) > 0:
            ref = lo
        elif f(hi) <= 0:
            ref = hi
        else:
            ref = optimize.brentq(f, lo, hi, xtol=1e-13, rtol=1e-15)
        err = abs(z64.reshape(-1)[perm[k]] - ref)
        worst = max(worst, err)
        assert err <= H.h, (k, err, H.h)
    print(f"growth matching vs continuous root: worst {worst:.2e} (h = {H.h:.2e})")


def test_unit_growth_reduces_to_plain_matching():
    n = 16
    J = inputs.make_intensity(n, 603).numpy()
    w = inputs.make_density(n, 604).numpy().astype(np.float32)
    H = oracle.History.from_params(7.95, 4.68, 2.90)
    ones = np.ones(H.T + 1)
    _, zg = oracle.zre_growth(J, w, H, ones)
    _, zp = oracle.zre(J, w, H, mode=oracle.CONTRACT)
    assert np.max(np.abs(zg - zp)) <= 1e-9


def test_defining_equation_holds_at_every_z():
    """For any z the cells with z_re > z hold the growth-weighted mass fraction
    x_i(z), to within one cell and the table interpolation."""
    n = 16
    J = inputs.make_intensity(n, 605, ties=False).numpy()
    w = inputs.make_density(n, 606).numpy().astype(np.float32)
    H = oracle.History.from_params(8.0, 4.0, 3.0)
    G = oracle.growth_table(H, 8.0)
    _, z64 = oracle.zre_growth(J, w, H, G)
    zf = z64.reshape(-1)
    wf = w.reshape(-1).astype(np.float64)
    N = zf.size
    d_mid = oracle.growth(8.0)
    for zz in np.linspace(H.a + 0.05, 13.0, 25):
        g = oracle.growth(zz) / d_mid
        mass = 1.0 + g * (wf - 1.0)
        frac = mass[zf > zz].sum() / mass.sum()
        xi = math.exp(-(((zz - H.a) / H.b) ** H.c))
        assert abs(frac - xi) <= np.max(np.abs(mass)) / mass.sum() + 1e-4, zz

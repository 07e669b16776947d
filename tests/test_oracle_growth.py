"""Pins of the oracle's growth-rescaled matching (Sec. 3.4.2 with
delta_m(z) = D(z)/D(z_mid) delta_m; readings G1, G2):

  * D(z) against a direct quadrature of the growing-mode integral of a flat
    matter + Lambda universe (an independent formula), its matter-dominated
    limit D = a and the matter-only case;
  * the node tables against that quadrature;
  * the Gauss-Legendre rule behind D: exact on monomials up to degree 2n - 1;
  * the matched z_re against a brute-force root of the continuous equation
    (scipy brentq on exact D and exact x_i, inside the first sign change found
    on a fine grid) on a small grid, within the node spacing h, also where
    some growth-weighted masses 1 + g delta are negative;
  * the bracket rule of reading G2 on a planted growth table whose gap changes
    sign three times: the walk stops at the first node with h_j > 0;
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


@pytest.mark.parametrize("z", [0.0, 0.3, 1.0, 3.0, 6.0, 8.0, 12.0, 30.0, 200.0])
@pytest.mark.parametrize("om", [0.3, 0.5, 0.1, 0.05])
def test_growth_matches_quadrature(z, om):
    assert oracle.growth(z, om) == pytest.approx(_growth_quad(z, om), rel=1e-13)


@pytest.mark.parametrize("n", [1, 2, 5, 16, 64])
def test_gauss_legendre_rule_is_exact_on_polynomials(n):
    x, w = oracle.gauss_legendre(n)
    assert np.all(np.diff(x) > 0) and np.all(w > 0)
    for k in range(2 * n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert np.sum(w * x ** k) == pytest.approx(exact, abs=1e-14), k
    ref_x, ref_w = np.polynomial.legendre.leggauss(n)   # the textbook table
    assert np.max(np.abs(x - ref_x)) <= 1e-14 and np.max(np.abs(w - ref_w)) <= 1e-14


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


def _first_crossing_root(f, lo, hi, grid=4000):
    """The lowest root of f on [lo, hi] where f turns from <= 0 to > 0: a fine
    grid finds the first positive sample, brentq refines inside that cell."""
    if f(lo) > 0:
        return lo
    zs = np.linspace(lo, hi, grid)
    prev = lo
    for z in zs[1:]:
        if f(z) > 0:
            return optimize.brentq(f, prev, z, xtol=1e-13, rtol=1e-15)
        prev = z
    return hi


@pytest.mark.parametrize("seed,wscale", [(601, 1.0), (611, 1.0), (621, 0.25)])
def test_brute_force_continuous_root(seed, wscale):
    """wscale < 1 makes many weights small (w < 0.12), so 1 + g delta < 0 for
    g > 1: the cells ranked last carry negative growth-weighted mass near a_w."""
    n = 8
    J = inputs.make_intensity(n, seed, ties=False, negatives=False).numpy()
    w = inputs.make_density(n, seed + 1).numpy().astype(np.float32)
    if wscale != 1.0:
        w = (w ** 3 * wscale).astype(np.float32)
        w = (w / w.mean()).astype(np.float32)
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

        ref = _first_crossing_root(f, H.a, H.z_top)
        err = abs(z64.reshape(-1)[perm[k]] - ref)
        worst = max(worst, err)
        assert err <= H.h, (k, err, H.h)
    g_max = oracle.growth(H.a) / d_mid
    neg = int(np.sum(1.0 + g_max * (w.astype(np.float64) - 1.0) < 0))
    if wscale != 1.0:
        assert neg > 0, "the case must hold cells with negative growth-weighted mass"
    print(f"growth matching vs continuous root: worst {worst:.2e} (h = {H.h:.2e}); "
          f"cells with 1 + g delta < 0 at a_w: {neg}")


def test_walk_stops_at_the_first_positive_gap():
    """A planted (non-physical) growth table makes the gap of every rank
    positive on two windows of nodes below its true root; the oracle's
    bracket must end at the first node with h_j > 0 (the lower window)."""
    n = 8
    J = inputs.make_intensity(n, 631, ties=False, negatives=False).numpy()
    w = inputs.make_density(n, 632).numpy().astype(np.float32)
    H = oracle.History.from_params(8.0, 4.0, 3.0)
    G = np.ones(H.T + 1)
    j1, j2 = 1000, 3000
    G[j1:j1 + 50] = 40.0       # a huge weight on the overdense ranks' mass
    G[j2:j2 + 50] = 40.0
    perm, C, Ctot = _masses(J, w)
    sel = np.arange(0, n ** 3, 3)
    zs, cells = oracle.zre_growth(J, w, H, G, ranks=sel)
    N = n ** 3
    X = H.X[: j2 + 200]     # every planted stop and every checked bracket lies below j2 + 200
    Gs = G[: j2 + 200]
    planted = 0
    for i, k in enumerate(sel):
        cnt = k + 1
        one = 1.0 - Gs
        h = (cnt * one + Gs * C[k]) / (N * one + Gs * Ctot) - X
        pos = np.nonzero(h > 0)[0]
        j = int(pos[0]) if pos.size else None
        if j is None:       # the first positive gap lies above the checked range: bracket above j2
            assert float(zs[i]) > H.a + (j2 + 199) * H.h
            continue
        if j == 0:
            ref = H.a
        else:
            t = -h[j - 1] / (h[j] - h[j - 1])
            ref = min((H.a + (j - 1) * H.h) + t * H.h, H.z_top)
        planted += int(j is not None and j in (j1, j2))
        assert cells[i] == perm[k]
        assert abs(float(zs[i]) - ref) <= 4e-6 * max(1.0, abs(ref)), (k, zs[i], ref)
    assert planted > 0, "some ranks must stop in a planted window"


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

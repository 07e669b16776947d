"""Growth-rescaled matching on the GPU (Sec. 3.4.2 with
delta_m(z) = D(z)/D(z_mid) delta_m; readings G1, G2) against the oracle.

Given identical intensities, weights, history table and growth table (the
library's growth table equals the oracle's byte for byte, checked on the CPU),
z_re must agree bit for bit.  At 1024^3 the defining equation is checked on
the device instead: for any z the cells with z_re > z hold the growth-weighted
mass fraction x_i(z) to within one cell.
"""
import math

import numpy as np
import pytest
import torch

import inputs
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amber():
    import paper_2109_10375_amd as amber
    assert torch.cuda.is_available()
    amber.lib()
    return amber


def _pair(amber, params, z_mid):
    H = oracle.History.from_params(*params)
    G = oracle.growth_table(H, z_mid)
    gh = amber.History.from_coeffs(H.a, H.b, H.c).with_growth(z_mid)
    return H, G, gh


@pytest.mark.parametrize("n,seed", [(16, 701), (32, 702), (64, 703), (128, 704)])
def test_growth_bitexact(amber, n, seed):
    J = inputs.make_intensity(n, seed).numpy()
    w = inputs.make_density(n, seed + 50).numpy().astype(np.float32)
    H, G, gh = _pair(amber, (8.0, 4.0, 3.0), 8.0)
    plan = amber.Plan(n, 1.0)
    (z,) = plan.zre(torch.from_numpy(J).cuda(), torch.from_numpy(w).cuda(), [gh])
    torch.cuda.synchronize()
    assert plan.status() == 0
    z32, _ = oracle.zre_growth(J, w, H, G)
    zg = z.cpu().numpy()
    print(f"growth n={n}: differing cells {int(np.sum(zg != z32))}", flush=True)
    assert np.array_equal(zg, z32)


def test_growth_mixed_with_plain_histories(amber):
    """One launch group holding growth and plain histories."""
    n = 64
    J = inputs.make_intensity(n, 711).numpy()
    w = inputs.make_density(n, 712).numpy().astype(np.float32)
    Hs = [oracle.History.from_params(*p) for p in ((7.95, 4.68, 2.90), (7.83, 6.54, 2.33))]
    plain = amber.History.from_coeffs(Hs[0].a, Hs[0].b, Hs[0].c)
    grown = amber.History.from_coeffs(Hs[1].a, Hs[1].b, Hs[1].c).with_growth(7.83)
    plan = amber.Plan(n, 1.0)
    z0, z1 = plan.zre(torch.from_numpy(J).cuda(), torch.from_numpy(w).cuda(), [plain, grown])
    torch.cuda.synchronize()
    ref0, _ = oracle.zre(J, w, Hs[0], mode=oracle.CONTRACT)
    ref1, _ = oracle.zre_growth(J, w, Hs[1], oracle.growth_table(Hs[1], 7.83))
    assert np.array_equal(z0.cpu().numpy(), ref0)
    assert np.array_equal(z1.cpu().numpy(), ref1)


def test_growth_1024_sampled_ranks_solve_their_equation(amber):
    """At 1024^3: for sampled ranks n, z_n solves m_n(z)/M(z) = x_i(z) with the
    growth-weighted masses (torch's stable sort and FP64 prefix sums) to within the
    node spacing h plus the FP32 rounding of z (brentq on the continuous
    equation, exact D and x_i)."""
    from scipy import optimize

    n = 1024
    dev = torch.device("cuda", 0)
    J = inputs.make_intensity(n, 721, device=dev)
    w = inputs.make_density(n, 722, device=dev, dtype=torch.float32).to(torch.float32).contiguous()
    H = oracle.History.from_params(8.0, 4.0, 3.0)
    gh = amber.History.from_coeffs(H.a, H.b, H.c).with_growth(8.0)
    plan = amber.Plan(n, 2000.0)
    (z,) = plan.zre(J, w, [gh])
    torch.cuda.synchronize()
    assert plan.status() == 0
    # the rank order from torch's stable sort (descending J, ties by index; -0 == +0)
    perm = torch.sort(J.reshape(-1), descending=True, stable=True).indices
    C = torch.cumsum(w.reshape(-1)[perm].to(torch.float64), 0)
    Ctot = float(C[-1])
    N = n ** 3
    rng = np.random.default_rng(9)
    ranks = np.concatenate([[0, 1, 2, 100, N // 2, N - 1], rng.integers(0, N, 60)])
    d_mid = oracle.growth(8.0)
    zs = z.reshape(-1)[perm[torch.from_numpy(ranks).to(dev)]].cpu().numpy().astype(np.float64)
    Cs = C[torch.from_numpy(ranks).to(dev)].cpu().numpy()
    worst = 0.0
    for r, zr, cn in zip(ranks, zs, Cs):
        k = float(r + 1)

        def f(zz):
            g = oracle.growth(zz) / d_mid
            return (k * (1 - g) + g * cn) / (N * (1 - g) + g * Ctot) - math.exp(-(((zz - H.a) / H.b) ** H.c))

        if f(H.a) > 0:
            ref = H.a
        elif f(H.z_top) <= 0:
            ref = H.z_top
        else:
            ref = optimize.brentq(f, H.a, H.z_top, xtol=1e-12, rtol=1e-15)
        worst = max(worst, abs(zr - ref))
        assert abs(zr - ref) <= H.h + 1e-6, (r, zr, ref)
    print(f"1024^3 growth matching, sampled ranks: worst |z - root| = {worst:.2e} (h = {H.h:.2e})", flush=True)

"""GPU parity of the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances:
  * rank order, z_re from identical intensities: bit-exact;
  * radiation J: relative L2 <= 1e-5 against the FP64 oracle, and every cell
    within 2e-5 of max|J| (FP32 FFT error, about log2(N^3) roundings of 6e-8);
  * end-to-end z_re (GPU radiation then GPU matching): every cell within 1e-4
    of the oracle's exact-mode match of the GPU's own FP32 intensity field;
    against the oracle's FP64 field every cell beyond 1e-4 is one whose exact
    ionized-mass fraction changed with the rank order (FP32 cannot resolve
    some nearly equal FP64 intensities), and their fraction is reported.
"""
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


def _oracle_hist(hist):
    return oracle.History.from_params(*hist)


def _gpu_hist(amber, H):
    return amber.History.from_coeffs(H.a, H.b, H.c)


# --------------------------------------------------------------- ranking ----

@pytest.mark.parametrize("n,seed", [(8, 1), (16, 2), (32, 3), (64, 4), (96, 5), (192, 6), (256, 7)])
def test_rank_bitexact_ties_zeros_negatives(amber, n, seed):
    print(f"rank n={n} seed={seed}", flush=True)
    J = inputs.make_intensity(n, seed)
    plan = amber.Plan(n, 1.0)
    perm = plan.rank(J.cuda())
    torch.cuda.synchronize()
    assert plan.status() == 0
    got = perm.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.rank(J.numpy()))


@pytest.mark.parametrize("kind", ["zeros", "sorted", "reversed", "two_values", "extremes"])
def test_rank_adversarial(amber, kind):
    n = 32
    n3 = n ** 3
    rng = np.random.default_rng(7)
    if kind == "zeros":
        J = np.where(rng.random(n3) < 0.5, np.float32(0.0), np.float32(-0.0)).astype(np.float32)
    elif kind == "sorted":
        J = np.arange(n3, dtype=np.float32)
    elif kind == "reversed":
        J = np.arange(n3, dtype=np.float32)[::-1].copy()
    elif kind == "two_values":
        J = np.where(rng.random(n3) < 0.3, np.float32(1.5), np.float32(-2.0)).astype(np.float32)
    else:
        vals = np.array([np.inf, -np.inf, 3.4e38, -3.4e38, 1e-45, -1e-45, 1e-38, 0.0, -0.0, 1.0],
                        dtype=np.float32)
        J = vals[rng.integers(0, vals.size, n3)]
    print(f"rank adversarial {kind}", flush=True)
    plan = amber.Plan(n, 1.0)
    perm = plan.rank(torch.from_numpy(J).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), oracle.rank(J))


def _few_bits_intensity(n, seed):
    """Intensities with at most 8 significant bits: the two low bytes of every
    sort key take one value, so the radix passes that split their input by
    those bytes' top bits find every key in one of their 8 segments."""
    rng = np.random.default_rng(seed)
    J = (rng.integers(1, 256, n ** 3) * np.exp2(rng.integers(-12, 12, n ** 3))).astype(np.float32)
    assert not np.any(J.view(np.uint32) & 0xFFFF)
    return J


def test_rank_one_segment_takes_all_tiles(amber):
    """All 4096 tiles of the second and third radix passes at 256^3 in one
    input segment: every block takes its tile from that segment after finding
    its own empty.  The permutation is still the oracle's, bit for bit."""
    n = 256
    print("rank one segment n=256", flush=True)
    J = _few_bits_intensity(n, 41)
    plan = amber.Plan(n, 1.0)
    perm = plan.rank(torch.from_numpy(J).cuda())
    torch.cuda.synchronize()
    assert plan.status() == 0
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), oracle.rank(J))


def test_zre_one_segment_takes_all_tiles(amber):
    """The same concentration on the weighted ranking that matching uses."""
    n = 128
    print("zre one segment n=128", flush=True)
    J = torch.from_numpy(_few_bits_intensity(n, 43).reshape(n, n, n))
    w = inputs.make_density(n, 44).to(torch.float32)
    H = _oracle_hist((8.0, 4.0, 3.0))
    plan = amber.Plan(n, 1.0)
    (z,) = plan.zre(J.cuda(), w.cuda(), [_gpu_hist(amber, H)])
    torch.cuda.synchronize()
    assert plan.status() == 0
    z_ref, _ = oracle.zre(J.numpy(), w.numpy(), H, mode=oracle.CONTRACT)
    assert np.array_equal(z.cpu().numpy(), z_ref)


def test_rank_nan_sets_status(amber):
    n = 16
    J = inputs.make_intensity(n, 3)
    J.view(-1)[77] = float("nan")
    plan = amber.Plan(n, 1.0)
    plan.rank(J.cuda())
    assert plan.status() & amber.STATUS_NAN_J


# -------------------------------------------------------------- matching ----

@pytest.mark.parametrize("n,seed", [(8, 11), (16, 12), (32, 13), (64, 14), (96, 15), (128, 16), (192, 17),
                                    (256, 18)])
def test_zre_bitexact_same_intensity(amber, n, seed):
    """Given identical J, w and history, GPU z_re equals the oracle's contract
    mode bit for bit."""
    print(f"zre n={n} seed={seed}", flush=True)
    J = inputs.make_intensity(n, seed)
    w = inputs.make_density(n, seed + 100).to(torch.float32)
    H = _oracle_hist((8.0, 4.0, 3.0))
    plan = amber.Plan(n, 1.0)
    (z,) = plan.zre(J.cuda(), w.cuda(), [_gpu_hist(amber, H)])
    torch.cuda.synchronize()
    assert plan.status() == 0
    z_ref, _ = oracle.zre(J.numpy(), w.numpy(), H, mode=oracle.CONTRACT)
    assert np.array_equal(z.cpu().numpy(), z_ref)


@pytest.mark.parametrize("n,kind", [(16, "ones"), (16, "wide"), (16, "subnormal"), (256, "wide"),
                                    (128, "subnormal")])
def test_zre_bitexact_edge_weights(amber, n, kind):
    """'wide' weights need the 128-bit exact sums; at 256^3 that path runs with
    the large sort tiles and the two-level scatter."""
    print(f"zre weights {kind} n={n}", flush=True)
    J = inputs.make_intensity(n, 21)
    w = inputs.make_weights_edge(n ** 3, 22, kind).reshape(n, n, n)
    H = _oracle_hist((7.83, 6.54, 2.33))
    plan = amber.Plan(n, 1.0)
    (z,) = plan.zre(J.cuda(), w.cuda(), [_gpu_hist(amber, H)])
    torch.cuda.synchronize()
    assert plan.status() == 0
    z_ref, _ = oracle.zre(J.numpy(), w.numpy(), H, mode=oracle.CONTRACT)
    assert np.array_equal(z.cpu().numpy(), z_ref)


def test_zre_several_histories_share_one_ranking(amber):
    n = 32
    J = inputs.make_intensity(n, 31)
    w = inputs.make_density(n, 32).to(torch.float32)
    hs = [(8.0, 4.0, 3.0), (7.95, 4.68, 2.90), (7.91, 5.45, 2.69), (7.83, 6.54, 2.33)]
    Hs = [_oracle_hist(h) for h in hs]
    plan = amber.Plan(n, 1.0)
    zs = plan.zre(J.cuda(), w.cuda(), [_gpu_hist(amber, H) for H in Hs])
    torch.cuda.synchronize()
    for z, H in zip(zs, Hs):
        z_ref, _ = oracle.zre(J.numpy(), w.numpy(), H, mode=oracle.CONTRACT)
        assert np.array_equal(z.cpu().numpy(), z_ref)


@pytest.mark.parametrize("n_hist", [4, 8])
def test_zre_histories_two_level_256(amber, n_hist):
    """256^3 takes the two-level scatter; with 4 histories the launch groups
    are 1 + 3 and with 8 they are 2 + 3 + 3: the last group's three histories
    share one second-level pass and one leaf pass in the rank-order buffers."""
    n = 256
    print(f"zre two-level n={n} histories={n_hist}", flush=True)
    J = inputs.make_intensity(n, 35)
    w = inputs.make_density(n, 36).to(torch.float32)
    hs = [(8.0, 4.0, 3.0), (7.95, 4.68, 2.90), (7.91, 5.45, 2.69), (7.83, 6.54, 2.33),
          (6.0, 2.0, 1.5), (10.0, 6.0, 4.0), (9.0, 3.0, 1.0), (7.0, 5.0, 2.0)][:n_hist]
    Hs = [_oracle_hist(h) for h in hs]
    plan = amber.Plan(n, 1.0)
    zs = plan.zre(J.cuda(), w.cuda(), [_gpu_hist(amber, H) for H in Hs])
    torch.cuda.synchronize()
    assert plan.status() == 0
    Jn, wn = J.numpy(), w.numpy()
    for k, (z, H) in enumerate(zip(zs, Hs)):
        z_ref, _ = oracle.zre(Jn, wn, H, mode=oracle.CONTRACT)
        diff = int(np.sum(z.cpu().numpy() != z_ref))
        print(f"  history {k}: differing cells {diff}", flush=True)
        assert diff == 0, k


@pytest.mark.parametrize("wide", [False, True])
def test_zre_exact_sum_width_boundary(amber, wide):
    """Weights whose exact total in units of the smallest ulp is just below
    2^64 (the 64-bit accumulators) or just above it (the 128-bit ones):
    32767 cells of weight 1 and one of 1.5 * 2^-26 (ulp 2^-49) give
    2^64 - 2^49 + 1.5 * 2^23; making two of the unit cells 2 gives
    2^64 + 2^50 + 1.5 * 2^23."""
    n = 32
    print(f"zre exact-sum width boundary, wide={wide}", flush=True)
    w = np.ones(n ** 3, dtype=np.float32)
    w[12345] = np.float32(1.5 * 2.0 ** -26)
    if wide:
        w[7] = 2.0
        w[30000] = 2.0
    J = inputs.make_intensity(n, 37)
    H = _oracle_hist((8.0, 4.0, 3.0))
    plan = amber.Plan(n, 1.0)
    (z,) = plan.zre(J.cuda(), torch.from_numpy(w.reshape(n, n, n)).cuda(), [_gpu_hist(amber, H)])
    torch.cuda.synchronize()
    assert plan.status() == 0
    total = sum(int(round(float(x) * 2.0 ** 49)) for x in w.tolist())
    assert (total >= 2 ** 64) == wide
    z_ref, _ = oracle.zre(J.numpy(), w.reshape(n, n, n), H, mode=oracle.CONTRACT)
    assert np.array_equal(z.cpu().numpy(), z_ref)


def test_status_is_sticky_until_read(amber):
    """A data error stays reported until amber_status reads it, whatever calls
    follow on the plan; reading clears it."""
    n = 16
    J = inputs.make_intensity(n, 3)
    Jbad = J.clone()
    Jbad.view(-1)[77] = float("nan")
    w = torch.ones(n, n, n).cuda()
    H = _gpu_hist(amber, _oracle_hist((8.0, 4.0, 3.0)))
    plan = amber.Plan(n, 1.0)
    assert plan.status() == 0
    plan.zre(Jbad.cuda(), w, [H])
    plan.zre(J.cuda(), w, [H])        # a clean call after the bad one
    plan.rank(J.cuda())
    assert plan.status() == amber.STATUS_NAN_J
    assert plan.status() == 0


def test_zre_rejects_inconsistent_table_geometry(amber):
    """amber_zre checks h, z_top and table_n against the coefficients on the
    host before anything runs."""
    import ctypes

    n = 16
    J = inputs.make_intensity(n, 5).cuda()
    w = torch.ones(n, n, n).cuda()
    H = _gpu_hist(amber, _oracle_hist((8.0, 4.0, 3.0)))
    plan = amber.Plan(n, 1.0)
    for field, value in (("table_n", 5), ("table_n", H.w.table_n + 1), ("h", H.w.h * 2), ("z_top", H.w.z_top + 1)):
        bad = amber.History.__new__(amber.History)
        bad.w = amber._lib.AmberWeibull.from_buffer_copy(H.w)
        bad.table = H.table
        setattr(bad.w, field, value)
        with pytest.raises(amber.AmberError) as e:
            plan.zre(J, w, [bad])
        assert e.value.code == amber._lib.E_ARG, field
    torch.cuda.synchronize()


def test_zre_more_histories_than_one_launch(amber):
    """Eight histories (the maximum) run in three launch groups; each result
    equals the oracle's and equals the same history run alone."""
    n = 16
    J = inputs.make_intensity(n, 33)
    w = inputs.make_density(n, 34).to(torch.float32)
    hs = [(8.0, 4.0, 3.0), (7.95, 4.68, 2.90), (7.91, 5.45, 2.69), (7.83, 6.54, 2.33),
          (6.0, 2.0, 1.5), (10.0, 6.0, 4.0), (9.0, 3.0, 1.0), (7.0, 5.0, 2.0)]
    Hs = [_oracle_hist(h) for h in hs]
    plan = amber.Plan(n, 1.0)
    G = [_gpu_hist(amber, H) for H in Hs]
    zs = plan.zre(J.cuda(), w.cuda(), G)
    torch.cuda.synchronize()
    assert plan.status() == 0
    for k, (z, H) in enumerate(zip(zs, Hs)):
        z_ref, _ = oracle.zre(J.numpy(), w.numpy(), H, mode=oracle.CONTRACT)
        assert np.array_equal(z.cpu().numpy(), z_ref), k
        (z1,) = plan.zre(J.cuda(), w.cuda(), [G[k]])
        assert torch.equal(z1, z)


def test_zre_bad_weights_set_status(amber):
    n = 16
    J = inputs.make_intensity(n, 41)
    H = _gpu_hist(amber, _oracle_hist((8.0, 4.0, 3.0)))
    plan = amber.Plan(n, 1.0)
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        w = torch.ones(n, n, n)
        w.view(-1)[123] = bad
        plan.zre(J.cuda(), w.cuda(), [H])
        assert plan.status() & amber.STATUS_BAD_W, bad
    w = torch.ones(n, n, n)
    w.view(-1)[5] = 1e-40
    w.view(-1)[6] = 3e38
    plan.zre(J.cuda(), w.cuda(), [H])
    assert plan.status() & amber.STATUS_RANGE
    plan.zre(J.cuda(), torch.ones(n, n, n).cuda(), [H])
    assert plan.status() == 0


# ------------------------------------------------------------- radiation ----

def _radiation_check(amber, n, L, l, S):
    plan = amber.Plan(n, L)
    (J,) = plan.radiation(S.cuda(), [l])
    torch.cuda.synchronize()
    J_ref = oracle.radiation(S.numpy().astype(np.float64), L, l)
    Jg = J.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(Jg - J_ref) / np.linalg.norm(J_ref)
    mx = np.max(np.abs(Jg - J_ref)) / np.max(np.abs(J_ref))
    print(f"radiation n={n} l={l}: relL2={rel:.2e} max={mx:.2e}", flush=True)
    assert rel <= 1e-5 and mx <= 2e-5
    return Jg, J_ref


@pytest.mark.parametrize("n", [8, 16, 32, 64, 96])
def test_radiation_random_source(amber, n):
    rng = np.random.default_rng(n)
    S = torch.from_numpy(rng.random((n, n, n)).astype(np.float32))
    _radiation_check(amber, n, 1.5625 * n, 3.0, S)


@pytest.mark.parametrize("n,l", [(32, 0.5), (64, 3.0), (64, 50.0), (128, 3.0)])
def test_radiation_halo_box(amber, n, l):
    cfg = inputs.BoxConfig("t", n, 1.5625 * n, max(2000, n ** 3 // 13), 1e9, 1e12, index=50 + n)
    w, S = inputs.make_box(cfg)
    _radiation_check(amber, n, cfg.box_len, l, S)


def test_radiation_point_source_and_sum_rule(amber):
    n, L, l = 64, 100.0, 3.0
    S = torch.zeros(n, n, n)
    S[3, 60, 17] = 1.0
    Jg, J_ref = _radiation_check(amber, n, L, l, S)
    assert abs(Jg.sum() - l) <= 1e-5 * l


def test_radiation_several_lmfp_share_one_forward(amber):
    n, L = 32, 50.0
    rng = np.random.default_rng(3)
    S = torch.from_numpy(rng.random((n, n, n)).astype(np.float32))
    ls = [0.5, 3.0, 20.0]
    plan = amber.Plan(n, L)
    Js = plan.radiation(S.cuda(), ls)
    torch.cuda.synchronize()
    for J, l in zip(Js, ls):
        (J1,) = plan.radiation(S.cuda(), [l])
        torch.cuda.synchronize()
        assert torch.equal(J, J1)
        J_ref = oracle.radiation(S.numpy().astype(np.float64), L, l)
        rel = np.linalg.norm(J.cpu().numpy() - J_ref) / np.linalg.norm(J_ref)
        assert rel <= 1e-5


# ------------------------------------------------------------ end to end ----

def test_end_to_end_config_64(amber):
    """64^3 box, 100 Mpc/h, 20000 halos, l_mfp = 3, history (8, 4, 3): GPU
    radiation + matching against the FP64 oracle end to end."""
    cfg = inputs.CONFIGS["c1"]
    w, S = inputs.make_box(cfg)
    H = _oracle_hist(cfg.histories[0])
    plan = amber.Plan(cfg.n, cfg.box_len)
    (J,) = plan.radiation(S.cuda(), [cfg.l_mfp[0]])
    (z,) = plan.zre(J, w.cuda(), [_gpu_hist(amber, H)])
    torch.cuda.synchronize()
    assert plan.status() == 0
    J_ref = oracle.radiation(S.numpy().astype(np.float64), cfg.box_len, cfg.l_mfp[0])
    Jg = J.cpu().numpy()
    rel = np.linalg.norm(Jg.astype(np.float64) - J_ref) / np.linalg.norm(J_ref)
    assert rel <= 1e-5
    zg = z.cpu().numpy().astype(np.float64)
    st = oracle.zre_per_cell_check(Jg, J_ref, w.numpy(), H, zg, tol=1e-4)
    print(f"e2e 64^3: J relL2={rel:.2e}; every cell within {st['max_err_same_field']:.2e} of the exact match "
          f"of the FP32 field; vs the FP64 field: {st['frac_within_tol_fp64']:.6f} within 1e-4, "
          f"{st['cells_over_tol_fp64']} beyond (max {st['max_err_fp64']:.2e}, all with a changed ionized-mass "
          f"fraction); max rank displacement {st['max_rank_displacement']}", flush=True)
    assert st["frac_within_tol_fp64"] >= 0.999
    pg = oracle.rank(Jg)
    # properties of the GPU result alone: the ionized mass fraction follows the
    # history (Sec. 3.4.2) and z_re is non-increasing along the GPU's rank order
    wf = w.numpy().reshape(-1).astype(np.float64)
    zf = zg.reshape(-1)
    for zz in np.linspace(H.a, 14.0, 120):
        frac = wf[zf > zz].sum() / wf.sum()
        xi = oracle.lib().oracle_weibull_x(zz, H.a, H.b, H.c)
        assert abs(frac - xi) <= wf.max() / wf.sum() + 1e-5
    assert np.all(np.diff(zf[pg]) <= 0)

"""FFT launch candidates and the tuner on the GPU (through the C-ABI).

Every compiled (column pass, z pass) candidate pair computes the same
radiation field (Sec. 3.4.1); they differ in FP32 rounding order only.
  * N = 128, 192, 256: every pair against the FP64 oracle on the whole field,
    with the bar of the radiation parity tests (relative L2 <= 1e-5, every
    cell within 2e-5 of max|J|);
  * N = 512 and 1024, where the oracle cannot run end to end: sampled DFT
    coefficients, DFT(J)_m = DFT(S)_m Khat(|k_m|), each computed one by one by
    the oracle in FP64, per-mode tolerance 1e-5 (|expected| + ||J||_2) as in
    the full-size test, with modes in the main half-spectrum and in the
    Nyquist plane; and, on every cell, agreement with the default pair within
    2e-5 relative L2 (both are within 1e-5 of the exact field).  At 1024 the
    pairs that vary one pass at a time are run: the column and z passes are
    separate kernels, so a pair is right when each of its passes is.
The tuner must time every pair, pick one, leave the plan on it and keep the
radiation bar; its cache must give the same pair to a new plan without timing.
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


def _pairs(amber, n, axes_only=False):
    cand = amber.fft_schedules(n)
    nc, nz = len(cand["col"]), len(cand["z"])
    if axes_only:
        return [(c, 0) for c in range(nc)] + [(0, z) for z in range(1, nz)]
    return [(c, z) for c in range(nc) for z in range(nz)]


@pytest.mark.parametrize("n", [128, 192, 256])
def test_every_schedule_matches_oracle(amber, n):
    rng = np.random.default_rng(1000 + n)
    S = rng.random((n, n, n)).astype(np.float32)
    L, l = 1.5625 * n, 3.0
    J_ref = oracle.radiation(S.astype(np.float64), L, l)
    ref_norm, ref_max = np.linalg.norm(J_ref), np.max(np.abs(J_ref))
    plan = amber.Plan(n, L)
    Sd = torch.from_numpy(S).cuda()
    pairs = _pairs(amber, n)
    assert len(pairs) > 1
    for c, z in pairs:
        plan.set_schedule(c, z)
        assert plan.schedule == (c, z)
        (J,) = plan.radiation(Sd, [l])
        torch.cuda.synchronize()
        Jg = J.cpu().numpy().astype(np.float64)
        rel = np.linalg.norm(Jg - J_ref) / ref_norm
        mx = np.max(np.abs(Jg - J_ref)) / ref_max
        print(f"n={n} schedule ({c},{z}): relL2={rel:.2e} max={mx:.2e}", flush=True)
        assert rel <= 1e-5 and mx <= 2e-5, (c, z)


_MODES = {
    512: [(0, 0, 0), (3, 5, 7), (300, 17, 255), (100, 400, 256), (256, 256, 256)],
    1024: [(0, 0, 0), (17, 200, 400), (1000, 900, 33), (511, 2, 512)],
}


@pytest.fixture(scope="module")
def big_box(request):
    cache = {}

    def get(n):
        if n not in cache:
            cache.clear()
            torch.cuda.empty_cache()
            cfg = inputs.CONFIGS["c3"] if n == 512 else inputs.CONFIGS["H"]
            w, S = inputs.make_box(cfg, device=torch.device("cuda", 0), dtype=torch.float32)
            del w
            Sh = S.cpu().numpy()
            smodes = {m: oracle.dft_coeff(Sh, m) for m in _MODES[n]}
            cache[n] = (cfg, S, smodes)
        return cache[n]
    return get


@pytest.mark.parametrize("n", [512, 1024])
def test_every_schedule_sampled_modes(amber, big_box, n):
    cfg, S, smodes = big_box(n)
    l = cfg.l_mfp[0]
    k0 = 2 * math.pi / cfg.box_len
    plan = amber.Plan(n, cfg.box_len)
    plan.set_schedule(0, 0)
    (J0,) = plan.radiation(S, [l])
    J = torch.empty_like(J0)
    for c, z in _pairs(amber, n, axes_only=(n == 1024)):
        plan.set_schedule(c, z)
        plan.radiation(S, [l], out=[J])
        torch.cuda.synchronize()
        d = torch.linalg.vector_norm((J - J0).double()) / torch.linalg.vector_norm(J0.double())
        Jh = J.cpu().numpy()
        jnorm = float(np.sqrt(np.sum(Jh.astype(np.float64) ** 2)))
        worst = 0.0
        for m, sm in smodes.items():
            s = [x if 2 * x <= n else x - n for x in m]
            expect = sm * oracle.kernel_hat(k0 * math.sqrt(sum(x * x for x in s)), l)
            err = abs(oracle.dft_coeff(Jh, m) - expect)
            worst = max(worst, err / (abs(expect) + jnorm))
            assert err <= 1e-5 * (abs(expect) + jnorm), (c, z, m)
        print(f"n={n} schedule ({c},{z}): vs default relL2={float(d):.2e}, worst mode err {worst:.2e}", flush=True)
        assert float(d) <= 2e-5, (c, z)
    del J, J0, plan
    torch.cuda.empty_cache()


def test_tuner_picks_a_pair_and_keeps_parity(amber):
    n, L, l = 128, 200.0, 3.0
    rng = np.random.default_rng(77)
    S = rng.random((n, n, n)).astype(np.float32)
    plan = amber.Plan(n, L)
    res = plan.tune(torch.from_numpy(S).cuda(), reps=2)
    cand = amber.fft_schedules(n)
    assert 0 <= res["col"] < len(cand["col"]) and 0 <= res["z"] < len(cand["z"])
    assert plan.schedule == (res["col"], res["z"])
    ms = np.array(res["ms"])
    assert ms.shape == (len(cand["col"]), len(cand["z"])) and np.all(np.isfinite(ms)) and np.all(ms > 0)
    # the chosen pair is the default, or beats it by the stated margin and is
    # the first pair within 1 % of the fastest
    c, z = res["col"], res["z"]
    if (c, z) != (0, 0):
        flat = ms.astype(np.float32).reshape(-1)      # the library compares in FP32
        beats = np.float32(0.98) * flat[0]
        near = np.float32(1.01) * flat.min()
        k = c * ms.shape[1] + z
        assert flat[k] < beats and flat[k] <= near
        assert not any(flat[j] < beats and flat[j] <= near for j in range(1, k))
    print(f"tuned n={n}: {res}", flush=True)
    (J,) = plan.radiation(torch.from_numpy(S).cuda(), [l])
    J_ref = oracle.radiation(S.astype(np.float64), L, l)
    rel = np.linalg.norm(J.cpu().numpy().astype(np.float64) - J_ref) / np.linalg.norm(J_ref)
    assert rel <= 1e-5


def test_tuner_cache_sets_the_same_pair_without_timing(amber, tmp_path):
    path = str(tmp_path / "fft_tune.json")
    p1 = amber.Plan(192, 300.0)
    first = amber.tune_plan(p1, reps=1, cache=path)
    assert not first["cached"]
    p2 = amber.Plan(192, 300.0)
    p2.set_schedule(len(amber.fft_schedules(192)["col"]) - 1, 0)
    second = amber.tune_plan(p2, reps=1, cache=path)
    assert second["cached"] and p2.schedule == (first["col"], first["z"])


def test_schedule_and_tuner_argument_errors(amber):
    plan = amber.Plan(64, 100.0)
    assert plan.schedule == (0, 0)
    with pytest.raises(amber.AmberError):
        plan.set_schedule(1, 0)          # 64 has one candidate per pass
    with pytest.raises(amber.AmberError):
        plan.set_schedule(0, -1)
    assert plan.schedule == (0, 0)
    S = torch.rand((64, 64, 64), device="cuda")
    with pytest.raises(amber.AmberError):
        plan.tune(S, reps=0)


def test_tuning_launches_are_not_traced(amber):
    """amber_plan_tune detaches an active profiler: after tuning, only the
    launches of the calls made outside the tuner are recorded."""
    n = 128
    plan = amber.Plan(n, 200.0)
    S = torch.rand((n, n, n), device="cuda")
    plan.profile_begin(256)
    plan.tune(S, reps=2)
    plan.radiation(S, [3.0])
    prof = plan.profile_end()
    assert prof["fft_z_r2c"][0] == 1 and prof["fft_z_c2r"][0] == 1 and prof["fft_x_mul"][0] == 1

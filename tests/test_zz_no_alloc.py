"""amber_zre_noalloc (amber_zre with the library's static scratch instead of
a workspace) against amber_zre, through the C-ABI: bit-identical z_re on two
calls in a row, the second on a smaller grid (the shared scratch keeps the
first call's contents), and the size limit."""
import ctypes

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


def test_noalloc_equals_workspace_call_twice_second_smaller(amber):
    cases = [(128, 901, [(8.0, 4.0, 3.0), (7.83, 6.54, 2.33)]), (64, 902, [(7.95, 4.68, 2.90)])]
    for n, seed, hp in cases:
        print(f"noalloc n={n} seed={seed} histories={len(hp)}", flush=True)
        Hs = [oracle.History.from_params(*p) for p in hp]
        gh = [amber.History.from_coeffs(H.a, H.b, H.c) for H in Hs]
        J = inputs.make_intensity(n, seed).cuda()
        w = inputs.make_density(n, seed + 1).to(torch.float32).cuda()
        plan = amber.Plan(n, 1.0)
        assert plan.workspace_bytes(1, len(hp)) <= amber._lib.NOALLOC_SCRATCH_BYTES
        ref = plan.zre(J, w, gh)
        out = [torch.full((n, n, n), -1.0, device="cuda") for _ in hp]
        got = plan.zre_noalloc(J, w, gh, out=out)
        torch.cuda.synchronize()
        assert plan.status() == 0
        for k, (a, b) in enumerate(zip(got, ref)):
            assert torch.equal(a, b), (n, k)
        z_or, _ = oracle.zre(J.cpu().numpy(), w.cpu().numpy(), Hs[0], mode=oracle.CONTRACT)
        assert np.array_equal(got[0].cpu().numpy(), z_or)


def test_noalloc_rejects_grids_beyond_its_scratch(amber):
    n = 256
    plan = amber.Plan(n, 1.0)
    H = oracle.History.from_params(8.0, 4.0, 3.0)
    gh = amber.History.from_coeffs(H.a, H.b, H.c)
    J = torch.zeros((n, n, n), device="cuda")
    with pytest.raises(amber.AmberError) as e:
        plan.zre_noalloc(J, torch.ones_like(J), [gh], out=[torch.empty_like(J)])
    assert e.value.code == amber._lib.E_SIZE

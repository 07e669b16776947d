"""Continuous-batching serving (paper_2109_10375_amd.serve): requests of
several grid sizes arrive together, are batched per grid size and run on
several streams at once, requests of one box merged into one batch item
(shared forward transform, one ranking per mean free path, a sparse set of
(l_mfp, history) outputs); every served J and z_re must equal, bit for bit,
the same request run alone through amber_radiation and amber_zre (reading B1:
a batch is the same work as its single calls).  The plain single-box path
(one request at a time) serves the same requests with the same results."""
import numpy as np
import pytest
import torch

import inputs

pytestmark = pytest.mark.gpu


def test_served_results_equal_each_request_alone():
    import paper_2109_10375_amd as amber
    from paper_2109_10375_amd import serve

    assert torch.cuda.is_available()
    dev = torch.device("cuda", 0)
    boxes = {}
    for n in (32, 64, 96):
        cfg = inputs.BoxConfig(f"serve.{n}", n, 1.953125 * n, max(500, n ** 3 // 40), 1e10, 1e12, index=900 + n)
        w, S = inputs.make_box(cfg, device=dev, dtype=torch.float32)
        boxes[n] = serve.Box(amber.Plan(n, cfg.box_len), S.contiguous(), w.contiguous())
    rng = np.random.default_rng(31)
    lmfp = (0.5, 3.0, 20.0)
    hists = ((8.0, 4.0, 3.0), (7.95, 4.68, 2.90), (7.83, 6.54, 2.33))
    # the requests arrive within a few hundred microseconds: they queue, merge and overlap
    reqs = [serve.Request(float(2e-5 * k), int(rng.choice([32, 64, 96])), float(rng.choice(lmfp)),
                          hists[int(rng.integers(0, 3))]) for k in range(18)]
    server = serve.Server(boxes, hbm_budget_bytes=1 << 30, max_batch=4, slots=3, exclusive_from=1 << 20)
    st = server.serve(reqs, keep_outputs=True)
    torch.cuda.synchronize()
    print(f"served {st['requests']} requests in {st['batches']} batches ({st['requests_merged']} merged), "
          f"at most {st['max_batches_in_flight']} in flight", flush=True)
    assert st["requests"] == len(reqs)
    assert st["max_batches_in_flight"] >= 2
    assert st["requests_merged"] >= 1
    # the largest grid run alone (the default), and the one-at-a-time path
    excl = serve.Server(boxes, hbm_budget_bytes=1 << 30, max_batch=4, slots=3)
    se = excl.serve(reqs, keep_outputs=True)
    fifo = serve.Server(boxes, hbm_budget_bytes=1 << 30, max_batch=1, slots=1, merge=False)
    sf = fifo.serve(reqs, keep_outputs=True)
    torch.cuda.synchronize()
    assert sf["batches"] == len(reqs) and sf["max_batches_in_flight"] == 1
    order = sorted(reqs, key=lambda r: r.t_arrival)
    for r, (J, z), (Je, ze), (Jf, zf) in zip(order, st["outputs"], se["outputs"], sf["outputs"]):
        assert torch.equal(J, Jf) and torch.equal(z, zf)
        assert torch.equal(J, Je) and torch.equal(z, ze)
        box = boxes[r.n]
        (Ja,) = box.plan.radiation(box.S, [r.l_mfp])
        (za,) = box.plan.zre(Ja, box.w, [amber.History.from_params(*r.history)])
        torch.cuda.synchronize()
        assert torch.equal(J, Ja), (r.n, r.l_mfp, r.history)
        assert torch.equal(z, za), (r.n, r.l_mfp, r.history)

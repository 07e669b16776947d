#!/usr/bin/env python
"""Throughput of the AMBER reionization-redshift hot path on one MI355X.

One step = amber_radiation (forward real FFT of the source field, multiply by
atan(k l_mfp)/k, inverse FFT) + amber_zre (rank, exact mass prefix, Weibull
inversion, scatter) over one synthetic box already resident in HBM.  The
default workload is the 1024^3 box (2000 Mpc/h, 80M halos on [1e10, 1e12]
Msun/h, l_mfp = 3 Mpc/h, history (z_mid, Delta_z, A_z) = (8, 4, 3)).

Prints one JSON line on stdout: grid cells/s over the timed steps, p50/p99 box
latency, the roofline of the dominant kernel (per-kernel HIP-event times taken
inside the timed region on the launch stream) and the FP64 CPU oracle timed on
a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

WORKLOADS = {
    "H": dict(cfg="H", desc="single box 1024^3, 2000 Mpc/h, 80M halos on [1e10,1e12] Msun/h, "
                            "l_mfp=3 Mpc/h, (z_mid, Delta_z, A_z)=(8, 4, 3)"),
    "H_growth": dict(cfg="H", growth=True,
                     desc="single box 1024^3 as the headline, matched with growth-rescaled overdensities "
                          "delta(z) = D(z)/D(z_mid) delta (flat LCDM, Omega_m = 0.3)"),
    "c2": dict(cfg="c2", desc="single box 256^3, 500 Mpc/h, 1.3M halos on [1e10,1e12] Msun/h, "
                             "l_mfp=3 Mpc/h, (z_mid, Delta_z, A_z)=(8, 4, 3)"),
    "c3": dict(cfg="c3", desc="512^3 box, 1000 Mpc/h, 10M halos; 8 l_mfp x 4 histories in one batch call "
                             "(1 forward FFT, 8 inverse, 8 rankings, 32 inversions)"),
    "c4": dict(cfg=None, desc="64 boxes, N uniform in {64,96,128,192,256}, L=1.953125 N, random l_mfp and history, "
                             "one batch call replayed as a HIP graph"),
    "H_halos": dict(cfg="H", desc="1024^3 box from its 80M-halo catalogue: CIC deposit on two interlaced meshes, "
                                  "deconvolution, radiation and matching (l_mfp=3, (8, 4, 3))"),
    "spectra": dict(cfg="H", desc="cross power spectrum of z_re (normalised redshift) and density (overdensity) "
                                  "of the 1024^3 box, 513 shells: two forward FFTs and the shell reduction"),
    "c5": dict(cfg=None, desc="Poisson requests at 20/s for 60 s, N in {128,256,512,1024} w.p. 0.4/0.3/0.2/0.1, "
                             "l_mfp and history from the 512^3 sweep sets; resident boxes, HBM-budget admission, "
                             "same-N batches admitted into free stream slots while others run (continuous batching)"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n: int) -> dict:
    """Bytes each kernel must move per launch (reads + writes of its operands)."""
    n3 = n ** 3
    half = n * n * (n // 2 + 1) * 8          # half spectrum, complex64
    main = n * n * (n // 2) * 8
    nyq = n * n * 8
    return {
        "fft_z_r2c": 4 * n3 + half,
        "fft_y": 2 * main,
        "fft_nyq_y": 2 * nyq,
        "fft_x_mul": 2 * main,
        "fft_nyq_x_mul": 2 * nyq,
        "fft_y_inv": 2 * main,
        "fft_nyq_y_inv": 2 * nyq,
        "fft_z_c2r": half + 4 * n3,
        "rank_hist": 4 * n3,
        "rank_pass0": 8 * n3 + 12 * n3,      # J, w in; key, index, w out
        "rank_pass1": 12 * n3 + 10 * n3,     # key's top 16 bits out
        "rank_pass2": 10 * n3 + 9 * n3,      # key's top 8 bits out
        "rank_pass3": 9 * n3 + 8 * n3,       # index, w out
        "match_tile_sums": 4 * n3,                 # sorted weights in
        "match_scan_partition": 8 * n3 + 8 * n3,   # rank order, w in; (cell, z) pairs out
        "match_partition2": 8 * n3 + 6 * n3,       # (cell, z) pairs in; (16-bit offset, z) out
        "match_leaf_scatter": 6 * n3 + 4 * n3,     # (offset, z) pairs in; z_re out
    }


# The survey's pass model of the 1024^3 pipeline (bytes per cell): FFT 5 passes of
# 8 B (3 forward + 3 inverse transforms with the x pair fused) = 40; radix sort:
# histogram 4 + digit passes 12 + 16 + 16 + 12 = 60 (key and index only); matching:
# rank order 4 + weight 4 + z_re 4 = 12.  The matching stage's 12 B are split
# here over its first and last kernels.  Nyquist-plane launches are part of
# their passes' bytes.
PASS_MODEL_BYTES_PER_CELL = {
    "fft_z_r2c": 8, "fft_y": 8, "fft_x_mul": 8, "fft_y_inv": 8, "fft_z_c2r": 8,
    "rank_hist": 4, "rank_pass0": 12, "rank_pass1": 16, "rank_pass2": 16, "rank_pass3": 12,
    "match_scan_partition": 8, "match_leaf_scatter": 4,
}
STAGES = (("fft", "fft_", 40), ("sort", "rank_", 60), ("match", "match_", 12))

KERNEL_SOURCES = {"fft_": "fft.hip", "rank_": "rank.hip", "match_": "match.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_box1024.txt")


def kernel_source_digest(name: str) -> str | None:
    """sha256 of the sources a library kernel is compiled from (its .hip file,
    the shared header and the build flags)."""
    import hashlib

    src = next((f for pre, f in KERNEL_SOURCES.items() if name.startswith(pre)), None)
    if src is None:
        return None
    pkg = os.path.join(ROOT, "paper_2109_10375_amd")
    h = hashlib.sha256()
    for f in (os.path.join(pkg, "csrc", src), os.path.join(pkg, "csrc", "internal.h"), os.path.join(pkg, "build.py")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name: str, n: int) -> tuple[float | None, str]:
    """HBM bytes per launch of `name` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel factor),
    or None when there is no entry or the kernel's sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter summary"
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            f = line.split()
            if len(f) >= 10 and f[0] == "kernel" and f[1] == name and int(f[3]) == n:
                if f[9] != kernel_source_digest(name):
                    return None, "kernel sources changed since the counters were taken"
                return float(f[5]) + float(f[7]), "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"
    return None, "no counter entry for this kernel"


def copy_peak_gbs(gib: int = 4, reps: int = 10) -> float:
    """Read + write bandwidth of a plain elementwise copy (torch.neg) of
    ``gib`` GiB: the practical HBM ceiling the kernels are compared with."""
    import torch

    x = torch.ones(gib * 2 ** 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        torch.neg(x, out=y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        torch.neg(x, out=y)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2 * gib * 2 ** 30 / (ms * 1e-3) / 1e9


def copy_calibration(mib: int) -> None:
    """A plain elementwise copy (negation) of `mib` MiB, three times: the known
    byte count against which the HBM counters are calibrated."""
    import torch

    src = torch.ones(mib * 2 ** 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: {mib} MiB read + {mib} MiB written per launch, 3 launches")


def cpu_baseline(sample_n: int, min_seconds: float, cfg=None) -> dict:
    import numpy as np

    import inputs
    import oracle

    oracle.lib()
    if cfg is None:
        cfg = inputs.BoxConfig("cpu", sample_n, 1.953125 * sample_n, max(1000, int(80e6 * (sample_n / 1024) ** 3)),
                               1e10, 1e12, index=7)
    w, S = inputs.make_box(cfg)
    S64 = S.numpy().astype(np.float64)
    wn = w.numpy()
    H = oracle.History.from_params(8.0, 4.0, 3.0)
    _ = H.X
    boxes = 0
    t0 = time.perf_counter()
    while True:
        J = oracle.radiation(S64, cfg.box_len, 3.0)
        oracle.zre(J, wn, H, mode=oracle.CONTRACT)
        boxes += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": boxes * sample_n ** 3 / el, "unit": "cells/s", "cores": oracle.num_threads(),
            "host": {"nproc": os.cpu_count(), "cpu": model, "omp_threads": oracle.num_threads(),
                     "note": "the radiation DFT loops use every thread; the rank order is one qsort"},
            "kind": "oracle",
            "sample": f"{boxes} box(es) of {sample_n}^3 (L={cfg.box_len:g} Mpc/h, l_mfp=3, (8,4,3)), "
                      f"FP64 naive-DFT radiation + qsort rank + exact-mass contract-mode matching, "
                      f"{el:.1f} s wall"}


def _common(args, metric: str, value: float, ms: float, desc: str, extra: dict) -> dict:
    out = {"metric": metric, "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": {"workload": desc}}
    out.update(extra)
    return out


def tune_fft(plan, S, args, known: dict | None = None) -> dict:
    """Sets the plan's FFT launch schedule: timed by the library's tuner on S
    (or read from --tune-cache), or the default pair with --no-tune.  `known`
    maps a grid size to a pair already chosen for another plan of that size."""
    import paper_2109_10375_amd as amber

    cand = amber.fft_schedules(plan.n)
    if args.no_tune:
        return {"col": list(cand["col"][0]), "z": list(cand["z"][0]), "tuned": False}
    if known is not None and plan.n in known:
        plan.set_schedule(*known[plan.n])
        c, z = known[plan.n]
        return {"col": list(cand["col"][c]), "z": list(cand["z"][z]), "tuned": True, "cached": True}
    t = time.perf_counter()
    res = amber.tune_plan(plan, S, reps=args.tune_reps, cache=args.tune_cache)
    if known is not None:
        known[plan.n] = (res["col"], res["z"])
    log(f"[bench] FFT schedule n={plan.n}: column (N1, C) = {tuple(res['col_split'])}, z (M1, ZL) = "
        f"{tuple(res['z_split'])}{' from the cache' if res['cached'] else ''} ({time.perf_counter() - t:.1f} s); "
        f"ms per radiation pass by [column][z] candidate: {[[round(x, 3) for x in row] for row in res['ms']]}")
    return {"col": res["col_split"], "z": res["z_split"], "tuned": True, "cached": res["cached"]}


def _time_steps(fn, steps: int, warmup: int):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        lat.append((a, b))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = sorted(x.elapsed_time(y) for x, y in lat)
    return el, ms


def _pct(ms, p):
    return ms[min(len(ms) - 1, max(0, int(round(p / 100.0 * (len(ms) - 1)))))]


def bench_sweep(args) -> dict:
    """512^3 box, 8 l_mfp x 4 histories: one batch call per step, and the same
    work as single calls (one radiation + one matching call per l_mfp)."""
    import torch

    import inputs
    import paper_2109_10375_amd as amber

    cfg = inputs.CONFIGS["c3"]
    dev = torch.device("cuda", 0)
    log(f"[bench] generating the {cfg.n}^3 box")
    w, S = inputs.make_box(cfg, device=dev, dtype=torch.float32)
    n, ls = cfg.n, list(cfg.l_mfp)
    plan = amber.Plan(n, cfg.box_len)
    sched = tune_fft(plan, S, args)
    hists = [amber.History.from_params(*h) for h in cfg.histories]
    J = [torch.empty((n, n, n), dtype=torch.float32, device=dev) for _ in ls]
    Z = [[torch.empty((n, n, n), dtype=torch.float32, device=dev) for _ in hists] for _ in ls]
    batch = amber.Batch([amber.BatchItem(plan, S, w, ls, J, hists, Z)])
    el, ms = _time_steps(batch.run, args.steps, args.warmup)
    if int(batch.status.sum()) != 0:
        raise RuntimeError("device status set")

    def serial():
        for li, l in enumerate(ls):
            plan.radiation(S, [l], out=[J[li]])
            plan.zre(J[li], w, hists, out=Z[li])

    el_s, ms_s = _time_steps(serial, args.steps, args.warmup)
    fields = args.steps * n ** 3 * len(ls)
    return _common(args, "J fields x cells/s (8 l_mfp x 4 histories per 512^3 box)", fields / el,
                   1e3 * el / args.steps, WORKLOADS["c3"]["desc"],
                   {"p50_ms": round(_pct(ms, 50), 3), "p99_ms": round(_pct(ms, 99), 3),
                    "serial_single_calls": {"value": fields / el_s, "ms_per_step": 1e3 * el_s / args.steps,
                                            "p50_ms": round(_pct(ms_s, 50), 3)},
                    "zre_fields_per_step": len(ls) * len(hists), "fft_schedule": sched})


def bench_mixed(args) -> dict:
    """64 boxes of mixed size in one batch, eager and as a replayed HIP graph,
    next to the same boxes as single calls."""
    import torch

    import inputs
    import paper_2109_10375_amd as amber

    dev = torch.device("cuda", 0)
    cfgs = inputs.c4_boxes(64)
    items, singles = [], []
    known, scheds = {}, {}
    log(f"[bench] generating {len(cfgs)} boxes")
    for cfg in cfgs:
        w, S = inputs.make_box(cfg, device=dev, dtype=torch.float32)
        n = cfg.n
        plan = amber.Plan(n, cfg.box_len)
        scheds[str(n)] = tune_fft(plan, S, args, known)
        h = amber.History.from_params(*cfg.histories[0])
        J = torch.empty((n, n, n), dtype=torch.float32, device=dev)
        z = torch.empty_like(J)
        items.append(amber.BatchItem(plan, S, w, list(cfg.l_mfp), [J], [h], [[z]]))
        singles.append((plan, S, w, cfg.l_mfp[0], J, h, z))
    batch = amber.Batch(items)
    cells = sum(c.n ** 3 for c in cfgs)
    el_e, ms_e = _time_steps(batch.run, args.steps, args.warmup)

    def capture(b):
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                b.run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        return g

    g1 = capture(batch)
    el_g1, ms_g1 = _time_steps(g1.replay, args.steps, args.warmup)
    lanes = amber.Batch(items, lanes=args.lanes)
    el_l, ms_l = _time_steps(lanes.run, args.steps, args.warmup)
    gl = capture(lanes)
    el_g, ms_g = _time_steps(gl.replay, args.steps, args.warmup)
    if int(batch.status.sum()) != 0 or int(lanes.status.sum()) != 0:
        raise RuntimeError("device status set")

    def serial():
        for plan, S, w, l, J, h, z in singles:
            plan.radiation(S, [l], out=[J])
            plan.zre(J, w, [h], out=[z])

    el_s, ms_s = _time_steps(serial, args.steps, args.warmup)
    return _common(args, "grid cells/s over a mixed batch of 64 boxes (HIP graph replay)",
                   args.steps * cells / el_g, 1e3 * el_g / args.steps, WORKLOADS["c4"]["desc"],
                   {"cells_per_step": cells, "sizes": sorted(collections.Counter(c.n for c in cfgs).items()),
                    "lanes": lanes.lanes,
                    "p50_ms": round(_pct(ms_g, 50), 3), "p99_ms": round(_pct(ms_g, 99), 3),
                    "eager_batch_lanes": {"value": args.steps * cells / el_l, "ms_per_step": 1e3 * el_l / args.steps},
                    "graph_one_lane": {"value": args.steps * cells / el_g1, "ms_per_step": 1e3 * el_g1 / args.steps},
                    "eager_batch_one_lane": {"value": args.steps * cells / el_e, "ms_per_step": 1e3 * el_e / args.steps},
                    "serial_single_calls": {"value": args.steps * cells / el_s,
                                            "ms_per_step": 1e3 * el_s / args.steps},
                    "speedup_vs_serial": round(el_s / el_g, 3),
                    "fft_schedule": scheds})


def bench_spectra(args) -> dict:
    """Two-point statistics of the 1024^3 box: P_zz, P_dd, P_zd, bias, r."""
    import torch

    import inputs
    import paper_2109_10375_amd as amber

    cfg = inputs.CONFIGS["H"]
    dev = torch.device("cuda", 0)
    w, S = inputs.make_box(cfg, device=dev, dtype=torch.float32)
    plan = amber.Plan(cfg.n, cfg.box_len)
    sched = tune_fft(plan, S, args)
    hist = amber.History.from_params(*cfg.histories[0])
    (J,) = plan.radiation(S, [cfg.l_mfp[0]])
    (z,) = plan.zre(J, w, [hist])
    del J, S
    torch.cuda.synchronize()
    st = {}

    def step():
        st["r"] = plan.spectra(z, w, kind_a=amber._lib.FIELD_REDSHIFT, kind_b=amber._lib.FIELD_OVERDENSITY,
                               n_bins=cfg.n // 2 + 1)

    el, ms = _time_steps(step, args.steps, args.warmup)
    r = st["r"]
    return _common(args, "grid cells/s of the z_re x density cross spectrum at 1024^3", args.steps * cfg.n ** 3 / el,
                   1e3 * el / args.steps, WORKLOADS["spectra"]["desc"],
                   {"p50_ms": round(_pct(ms, 50), 3), "p99_ms": round(_pct(ms, 99), 3),
                    "r_zd_at_k": {f"{float(r['k'][i]):.4f}": round(float(r["r"][i]), 4) for i in (1, 4, 16, 64, 256)},
                    "b_zd_at_k": {f"{float(r['k'][i]):.4f}": round(float(r["bias"][i]), 4) for i in (1, 4, 16, 64, 256)},
                    "fft_schedule": sched})


def bench_halos(args) -> dict:
    """The headline box built from its halo catalogue on the GPU each step."""
    import torch

    import inputs
    import paper_2109_10375_amd as amber

    cfg = inputs.CONFIGS["H"]
    dev = torch.device("cuda", 0)
    n = cfg.n
    w = inputs.make_density(n, inputs.config_seed(cfg.index, 0), device=dev, dtype=torch.float32).to(torch.float32)
    pos, mass = inputs.make_halos(cfg, device=dev, w=w)
    plan = amber.Plan(n, cfg.box_len)
    sched = tune_fft(plan, w, args)   # any N^3 field times the same passes
    hist = amber.History.from_params(*cfg.histories[0])
    J = torch.empty((n, n, n), dtype=torch.float32, device=dev)
    z = torch.empty_like(J)

    def step():
        plan.radiation_from_halos(pos, mass, [cfg.l_mfp[0]], scheme=amber._lib.ASSIGN_CIC, interlace=True, out=[J])
        plan.zre(J, w, [hist], out=[z])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.profile_begin(64 * args.steps)
    el, ms = _time_steps(step, args.steps, 0)
    prof = plan.profile_end()
    return _common(args, "grid cells/s from a halo catalogue (deposit + radiation + zre match) at 1024^3",
                   args.steps * n ** 3 / el, 1e3 * el / args.steps, WORKLOADS["H_halos"]["desc"],
                   {"p50_ms": round(_pct(ms, 50), 3), "p99_ms": round(_pct(ms, 99), 3), "n_halo": cfg.n_halo,
                    "kernels_ms_per_step": {k: round(t / args.steps, 4)
                                            for k, (c, t) in sorted(prof.items(), key=lambda kv: -kv[1][1])},
                    "fft_schedule": sched})


def bench_serving(args) -> dict:
    """Poisson request stream served from resident boxes."""
    import torch

    import inputs
    import paper_2109_10375_amd as amber
    from paper_2109_10375_amd import serve

    dev = torch.device("cuda", 0)
    boxes, scheds = {}, {}
    for n in (128, 256, 512, 1024):
        cfg = inputs.BoxConfig(f"c5.{n}", n, 1.953125 * n, max(1000, int(1.3e6 * (n / 256) ** 3)), 1e10, 1e12,
                               index=200 + n)
        log(f"[bench] generating the resident {n}^3 box")
        w, S = inputs.make_box(cfg, device=dev, dtype=torch.float32)
        boxes[n] = serve.Box(amber.Plan(n, cfg.box_len), S, w)
        scheds[str(n)] = tune_fft(boxes[n].plan, S, args)
    server = serve.Server(boxes, hbm_budget_bytes=args.hbm_budget_gb * 2 ** 30, max_batch=16, slots=args.serve_slots)
    warm = serve.requests_from(inputs.c5_requests(2.0, seed=55))
    server.serve(warm)
    reqs = serve.requests_from(inputs.c5_requests(args.serve_seconds))
    offered = sum(r.n ** 3 for r in reqs) / args.serve_seconds
    log(f"[bench] serving {len(reqs)} requests ({offered / 1e9:.2f} G cells/s offered)")
    st = server.serve(reqs)
    log(f"[bench] served: {st['requests']} requests in {st['batches']} batches ({st['requests_merged']} merged), "
        f"p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms")
    # the plain single-box path on the same arrivals: one request at a time, in arrival order
    hists = server.hists
    server = None                      # its per-slot workspaces
    torch.cuda.empty_cache()
    fifo = serve.Server(boxes, hbm_budget_bytes=args.hbm_budget_gb * 2 ** 30, max_batch=1, slots=1, merge=False)
    fifo.hists = hists
    sf = fifo.serve(reqs)
    log(f"[bench] one at a time: p50 {sf['p50_ms']:.1f} ms, p99 {sf['p99_ms']:.1f} ms")
    # the same requests back to back on one stream, device time only (no arrivals, no queueing)
    outs = {n: (torch.empty((n, n, n), dtype=torch.float32, device=dev),
                torch.empty((n, n, n), dtype=torch.float32, device=dev)) for n in boxes}
    serial_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        b = boxes[r.n]
        J, z = outs[r.n]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.plan.radiation(b.S, [r.l_mfp], out=[J])
        b.plan.zre(J, b.w, [fifo.history(r.history)], out=[z])
        e1.record()
        serial_ms.append((e0, e1))
    torch.cuda.synchronize()
    serial_el = time.perf_counter() - t0
    serial_lat = sorted(a.elapsed_time(b_) for a, b_ in serial_ms)
    del outs
    log(f"[bench] back to back: {len(reqs)} requests in {serial_el:.2f} s")
    return _common(args, "served grid cells/s (Poisson requests, p50/p99 latency)", st["cells_per_s_busy"],
                   1e3 * st["busy_s"] / max(1, st["batches"]), WORKLOADS["c5"]["desc"],
                   {"p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                    "mean_latency_ms": round(st["mean_ms"], 3), "requests": st["requests"],
                    "batches": st["batches"], "requests_merged": st["requests_merged"],
                    "p50_ms_by_n": st["p50_ms_by_n"], "p99_ms_by_n": st["p99_ms_by_n"],
                    "offered_cells_per_s": offered,
                    "makespan_s": round(st["makespan_s"], 3), "busy_s": round(st["busy_s"], 3),
                    "slots": st["slots"], "max_batches_in_flight": st["max_batches_in_flight"],
                    "hbm_budget_gb": args.hbm_budget_gb, "arrivals_s": args.serve_seconds,
                    "single_box_path_same_arrivals": {
                        "value": sf["cells_per_s_busy"], "p50_ms": round(sf["p50_ms"], 3),
                        "p99_ms": round(sf["p99_ms"], 3), "mean_latency_ms": round(sf["mean_ms"], 3),
                        "p99_ms_by_n": sf["p99_ms_by_n"], "busy_s": round(sf["busy_s"], 3)},
                    "serial_back_to_back": {"value": st["cells"] / serial_el, "seconds": round(serial_el, 3),
                                            "device_p50_ms": round(_pct(serial_lat, 50), 3),
                                            "device_p99_ms": round(_pct(serial_lat, 99), 3)},
                    "fft_schedule": scheds})


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="H", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=128)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="c5: seconds of Poisson arrivals")
    ap.add_argument("--hbm-budget-gb", type=int, default=96, help="c5: HBM for outputs of requests in flight")
    ap.add_argument("--serve-slots", type=int, default=2, help="c5: streams with batches in flight at once")
    ap.add_argument("--lanes", type=int, default=4, help="c4: concurrent streams the batch's boxes are dealt to")
    ap.add_argument("--no-tune", action="store_true", help="keep the default FFT schedule (no autotuning)")
    ap.add_argument("--tune-reps", type=int, default=5, help="timed radiation passes per schedule pair and round")
    ap.add_argument("--tune-cache", default=None, metavar="JSON",
                    help="schedule cache keyed by device and grid size (default: tune in this process)")
    ap.add_argument("--cpu-only", default=None, metavar="N[,N...]",
                    help="time only the CPU oracle on boxes of these sizes (64 is the c1 box) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain copy of MIB MiB (for HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2

    if args.cpu_only:
        import inputs
        for n in [int(x) for x in args.cpu_only.split(",")]:
            res = cpu_baseline(n, args.cpu_seconds, inputs.CONFIGS["c1"] if n == 64 else None)
            print(json.dumps({"cpu_only": True, "n": n, "cpu_baseline": res}), flush=True)
        return 0

    import torch

    import inputs
    import paper_2109_10375_amd as amber

    amber.lib()  # raises when the HIP library is missing: there is no fallback
    if args.workload in ("c3", "c4", "c5", "spectra", "H_halos"):
        torch.cuda.set_device(0)
        out = {"c3": bench_sweep, "c4": bench_mixed, "c5": bench_serving, "spectra": bench_spectra,
               "H_halos": bench_halos}[args.workload](args)
        print(json.dumps(out), flush=True)
        return 0
    wl = WORKLOADS[args.workload]
    cfg = inputs.CONFIGS[wl["cfg"]]
    n, n3 = cfg.n, cfg.n ** 3
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    log(f"[bench] generating {cfg.name} inputs on the GPU ({cfg.notes})")
    tg = time.perf_counter()
    w, S = inputs.make_box(cfg, device=dev, dtype=torch.float32)
    torch.cuda.synchronize()
    log(f"[bench] inputs ready in {time.perf_counter() - tg:.1f} s")

    plan = amber.Plan(n, cfg.box_len)
    sched = tune_fft(plan, S, args)
    hist = amber.History.from_params(*cfg.histories[0])
    if wl.get("growth"):
        hist = hist.with_growth(cfg.histories[0][0])
    J = torch.empty((n, n, n), dtype=torch.float32, device=dev)
    z = torch.empty((n, n, n), dtype=torch.float32, device=dev)
    plan.workspace(1)
    l_mfp = [cfg.l_mfp[0]]

    def step():
        plan.radiation(S, l_mfp, out=[J])
        plan.zre(J, w, [hist], out=[z])

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    st = plan.status()
    if st:
        raise RuntimeError(f"device status {st} after warmup")

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    plan.profile_begin(64 * args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record()
        step()
        ends[k].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_end()
    lat = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    elapsed = t1 - t0
    value = args.steps * n3 / elapsed

    def pct(p):
        i = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[i]

    copy_gbs = copy_peak_gbs()
    alg = algorithmic_bytes(n)
    rows = []
    for name, (launches, tot_ms) in prof.items():
        avg = tot_ms / launches
        b = alg.get(name)
        gbs = b / (avg * 1e-3) / 1e9 if b else None
        rows.append((tot_ms, name, launches, avg, b, gbs))
    rows.sort(reverse=True)
    log(f"[bench] {'kernel':22s} {'launches':>8s} {'avg ms':>9s} {'share':>6s} {'alg GB':>8s} {'GB/s':>8s} {'%HBM':>6s}")
    tot_all = sum(r[0] for r in rows)
    for tot_ms, name, launches, avg, b, gbs in rows:
        log(f"[bench] {name:22s} {launches:8d} {avg:9.3f} {100 * tot_ms / tot_all:5.1f}% "
            f"{(b or 0) / 1e9:8.2f} {gbs or 0:8.0f} {100 * (gbs or 0) / HBM_PEAK_GBS:5.1f}")
    # the dominant kernel (largest share of the step) against the survey's pass-model bytes
    dom = next(r for r in rows if r[1] in PASS_MODEL_BYTES_PER_CELL)
    pm_bytes = PASS_MODEL_BYTES_PER_CELL[dom[1]] * n3
    pm_gbs = pm_bytes / (dom[3] * 1e-3) / 1e9
    traffic, traffic_src = measured_traffic(dom[1], n)
    roof = {"bound": "hbm", "kernel": dom[1], "achieved": round(pm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(pm_gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": traffic_src,
            "bytes_model": "survey pass model (FFT 40, sort 60, matching 12 B per cell)",
            "algorithmic_bytes_per_launch": pm_bytes, "avg_launch_ms": round(dom[3], 4),
            "design_bytes_per_launch": dom[4],
            "design_frac": round((dom[5] or 0) / HBM_PEAK_GBS, 4)}
    stages = {}
    step_ms = 1e3 * elapsed / args.steps
    for stage, prefix, model_b in STAGES:
        ks = [r for r in rows if r[1].startswith(prefix)]
        ms = sum(r[0] for r in ks) / args.steps
        design_b = sum(alg.get(r[1], 0) * r[2] for r in ks) / args.steps
        kc = [r for r in ks if r[1] in alg]
        counted = [measured_traffic(r[1], n)[0] for r in kc]
        counter_b = (sum(c * r[2] for c, r in zip(counted, kc)) / args.steps
                     if kc and all(c is not None for c in counted) else None)
        gbs = model_b * n3 / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        stages[stage] = {"ms_per_step": round(ms, 3), "share": round(ms / step_ms, 4),
                         "pass_model_bytes_per_cell": model_b, "pass_model_gbs": round(gbs, 1),
                         "pass_model_frac": round(gbs / HBM_PEAK_GBS, 4),
                         "design_bytes_per_cell": round(design_b / n3, 2),
                         "design_frac": round(design_b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else 0.0,
                         "counter_bytes_per_cell": round(counter_b / n3, 2) if counter_b is not None else None,
                         "kernels": [r[1] for r in ks]}
        log(f"[bench] stage {stage:5s}: {ms:7.3f} ms/step, pass model {model_b} B/cell -> {gbs:7.0f} GB/s "
            f"({100 * gbs / HBM_PEAK_GBS:4.1f}% of HBM); design {design_b / n3:5.1f} B/cell; counters "
            f"{'n/a' if counter_b is None else f'{counter_b / n3:5.1f} B/cell'}")
    pipe_bytes = sum(alg[r[1]] * r[2] for r in rows if r[1] in alg) / args.steps
    out = {
        "metric": "grid cells/s (radiation FFT-convolve + zre match) at 1024^3; p50/p99 box latency",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "box_len": cfg.box_len, "n_halo": cfg.n_halo,
                   "l_mfp": l_mfp[0], "history": list(cfg.histories[0]),
                   "precision": "FFT f32; mass prefix exact int128; F and inversion f64",
                   "fft_schedule": sched},
        "p50_ms": round(pct(50), 3),
        "p99_ms": round(pct(99), 3),
        "pipeline_alg_bytes_per_step": pipe_bytes,
        "pipeline_frac_hbm": round(pipe_bytes / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
        # the fixed pass model of the pipeline (FFT 40 + sort 60 + scan 12 bytes per cell) and the
        # compulsory I/O (S, J twice, w, z: 20 bytes per cell), against the spec and a measured copy
        "pass_model_frac_hbm": round(112 * n3 / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
        "compulsory_io_frac_hbm": round(20 * n3 / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
        "copy_peak_gbs": round(copy_gbs, 1),
        "pass_model_frac_copy": round(112 * n3 / (elapsed / args.steps) / 1e9 / copy_gbs, 4),
        "roofline": roof,
        "stages": stages,
        "kernels_ms_per_step": {r[1]: round(r[0] / args.steps, 4) for r in rows},
    }
    del J, z, w, S
    plan = None
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log(f"[bench] timing the FP64 CPU oracle on {args.cpu_sample_n}^3 boxes")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

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
    "c2": dict(cfg="c2", desc="single box 256^3, 500 Mpc/h, 1.3M halos on [1e10,1e12] Msun/h, "
                             "l_mfp=3 Mpc/h, (z_mid, Delta_z, A_z)=(8, 4, 3)"),
    "c3": dict(cfg="c3", desc="single box 512^3, 1000 Mpc/h, 10M halos, l_mfp=3, (8, 4, 3)"),
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
        "rank_pass1": 12 * n3 + 12 * n3,
        "rank_pass2": 12 * n3 + 12 * n3,
        "rank_pass3": 12 * n3 + 8 * n3,      # index, w out
        "match_tile_sums": 4 * n3,                 # sorted weights in
        "match_scan_partition": 8 * n3 + 8 * n3,   # rank order, w in; (cell, z) pairs out
        "match_partition2": 8 * n3 + 8 * n3,       # (cell, z) pairs in and out
        "match_leaf_scatter": 8 * n3 + 4 * n3,     # (cell, z) pairs in; z_re out
    }


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


def cpu_baseline(sample_n: int, min_seconds: float) -> dict:
    import numpy as np

    import inputs
    import oracle

    oracle.lib()
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
    return {"value": boxes * sample_n ** 3 / el, "unit": "cells/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{boxes} box(es) of {sample_n}^3 (L={cfg.box_len:g} Mpc/h, l_mfp=3, (8,4,3)), "
                      f"FP64 naive-DFT radiation + qsort rank + exact-mass contract-mode matching, "
                      f"{el:.1f} s wall"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="H", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=128)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain copy of MIB MiB (for HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2

    import torch

    import inputs
    import paper_2109_10375_amd as amber

    amber.lib()  # raises when the HIP library is missing: there is no fallback
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
    hist = amber.History.from_params(*cfg.histories[0])
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
    dom = next(r for r in rows if r[4])
    traffic, traffic_src = measured_traffic(dom[1], n)
    roof = {"bound": "hbm", "kernel": dom[1], "achieved": round(dom[5], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(dom[5] / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": traffic_src,
            "algorithmic_bytes_per_launch": dom[4], "avg_launch_ms": round(dom[3], 4)}
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
                   "precision": "FFT f32; mass prefix exact int128; F and inversion f64"},
        "p50_ms": round(pct(50), 3),
        "p99_ms": round(pct(99), 3),
        "pipeline_alg_bytes_per_step": pipe_bytes,
        "pipeline_frac_hbm": round(pipe_bytes / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roof,
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

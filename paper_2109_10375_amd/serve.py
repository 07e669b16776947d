"""Serving z_re requests on one GPU.

A request asks for the z_re field of a resident box (one per grid size) under
its own mean free path and history.  The server keeps the input fields and one
workspace per grid size resident in HBM, admits queued requests while the
outputs of a batch fit an HBM budget, batches requests of the same grid size
into one amber_batch_run call, and reports per-request latency.

Arrivals follow a given schedule on a virtual clock; service times are the
measured device times of the batches (the clock jumps over idle gaps instead of
waiting for them).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, Iterable, List, Sequence, Tuple

import torch

from . import _lib


@dataclasses.dataclass
class Request:
    t_arrival: float          # seconds on the virtual clock
    n: int                    # grid size of the resident box
    l_mfp: float
    history: Tuple[float, float, float]   # (z_mid, Delta_z, A_z)


@dataclasses.dataclass
class Box:
    plan: _lib.Plan
    S: torch.Tensor           # source field, N^3 FP32, resident
    w: torch.Tensor           # gas-mass weights, N^3 FP32, resident


def output_bytes(n: int) -> int:
    """HBM a request holds while it is served: its J and z_re fields."""
    return 8 * n ** 3


class Server:
    def __init__(self, boxes: Dict[int, Box], hbm_budget_bytes: int, max_batch: int = 16):
        self.boxes = boxes
        self.budget = int(hbm_budget_bytes)
        self.max_batch = int(max_batch)
        self.hists: Dict[Tuple[float, float, float], _lib.History] = {}
        self.ws: Dict[int, torch.Tensor] = {}
        for n, box in boxes.items():
            if output_bytes(n) > self.budget:
                raise ValueError(f"HBM budget {self.budget} B cannot hold one {n}^3 request")
            self.ws[n] = box.plan.workspace(1)

    def history(self, params: Tuple[float, float, float]) -> _lib.History:
        h = self.hists.get(params)
        if h is None:
            h = self.hists[params] = _lib.History.from_params(*params)
        return h

    def _run(self, batch: List[Request]) -> None:
        n = batch[0].n
        box = self.boxes[n]
        items = []
        for r in batch:
            J = torch.empty((n, n, n), dtype=torch.float32, device=box.S.device)
            z = torch.empty_like(J)
            items.append(_lib.BatchItem(box.plan, box.S, box.w, [r.l_mfp], [J], [self.history(r.history)], [[z]]))
        b = _lib.Batch(items, ws=self.ws[n])
        b.run()
        torch.cuda.synchronize()
        if int(b.status.abs().sum()) != 0:
            raise RuntimeError(f"device status {b.status.tolist()} in a batch of {n}^3 requests")

    def serve(self, requests: Iterable[Request]) -> dict:
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        for r in pending:            # fit every history before the clock starts
            self.history(r.history)
        queue: List[Request] = []
        clock, busy = 0.0, 0.0
        lat: List[float] = []
        cells = 0
        batches = 0
        while pending or queue:
            if not queue and pending[0].t_arrival > clock:
                clock = pending[0].t_arrival
            while pending and pending[0].t_arrival <= clock:
                queue.append(pending.popleft())
            n = queue[0].n           # the oldest request decides the grid size
            batch, used = [], 0
            for r in queue:
                if r.n != n:
                    continue
                if len(batch) >= self.max_batch or used + output_bytes(n) > self.budget:
                    break
                batch.append(r)
                used += output_bytes(n)
            chosen = set(map(id, batch))
            queue = [r for r in queue if id(r) not in chosen]
            t0 = time.perf_counter()
            self._run(batch)
            dt = time.perf_counter() - t0
            clock += dt
            busy += dt
            batches += 1
            for r in batch:
                lat.append(clock - r.t_arrival)
                cells += r.n ** 3
        lat.sort()

        def pct(p: float) -> float:
            return lat[min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))]

        return {"requests": len(lat), "batches": batches, "cells": cells, "busy_s": busy, "makespan_s": clock,
                "cells_per_s_busy": cells / busy if busy > 0 else 0.0,
                "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99), "mean_ms": 1e3 * sum(lat) / len(lat)}


def requests_from(schedule: Sequence[Tuple[float, int, float, Tuple[float, float, float]]]) -> List[Request]:
    return [Request(t, n, l, tuple(h)) for t, n, l, h in schedule]

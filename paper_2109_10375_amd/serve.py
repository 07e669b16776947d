"""Serving z_re requests on one GPU with continuous batching.

A request asks for the z_re field of a resident box (one per grid size) under
its own mean free path and history.  The server keeps the input fields
resident in HBM and runs a fixed number of slots, each a HIP stream with its
own workspace per grid size.  Requests arrive on the wall clock; whenever a
slot is free and the outputs fit the HBM budget, the queued requests of the
oldest request's grid size are taken as one batch (one amber_batch_run) and
launched on that slot, so batches keep being admitted while others are still
on the device and the work of different slots overlaps.  Completion is seen
through an event per batch; a request's latency runs from its arrival to the
moment its batch is seen complete.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import torch

from . import _lib


@dataclasses.dataclass
class Request:
    t_arrival: float          # seconds after the start of serve()
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


@dataclasses.dataclass
class _InFlight:
    batch: List[Request]
    job: _lib.Batch
    outputs: List[Tuple[torch.Tensor, torch.Tensor]]
    done: torch.cuda.Event
    t_launch: float
    bytes: int


class Server:
    def __init__(self, boxes: Dict[int, Box], hbm_budget_bytes: int, max_batch: int = 16, slots: int = 2):
        if slots < 1:
            raise ValueError("at least one slot")
        self.boxes = boxes
        self.budget = int(hbm_budget_bytes)
        self.max_batch = int(max_batch)
        self.hists: Dict[Tuple[float, float, float], _lib.History] = {}
        device = next(iter(boxes.values())).S.device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]  # default priority
        self.ws: List[Dict[int, torch.Tensor]] = [dict() for _ in range(slots)]
        for n, box in boxes.items():
            if output_bytes(n) > self.budget:
                raise ValueError(f"HBM budget {self.budget} B cannot hold one {n}^3 request")
            probe = _lib.BatchItem(box.plan, box.S, box.w, [1.0], [box.S], [self.history((8.0, 4.0, 3.0))],
                                   [[box.w]])
            need = _lib.Batch.workspace_bytes([probe])
            for k in range(slots):
                self.ws[k][n] = torch.empty(need, dtype=torch.uint8, device=device)

    def history(self, params: Tuple[float, float, float]) -> _lib.History:
        h = self.hists.get(params)
        if h is None:
            h = self.hists[params] = _lib.History.from_params(*params)
        return h

    def _launch(self, slot: int, batch: List[Request], now: float) -> _InFlight:
        n = batch[0].n
        box = self.boxes[n]
        stream = self.streams[slot]
        items, outputs = [], []
        for r in batch:
            J = torch.empty((n, n, n), dtype=torch.float32, device=box.S.device)
            z = torch.empty_like(J)
            outputs.append((J, z))
            items.append(_lib.BatchItem(box.plan, box.S, box.w, [r.l_mfp], [J], [self.history(r.history)], [[z]]))
        job = _lib.Batch(items, ws=self.ws[slot][n])
        stream.wait_stream(torch.cuda.current_stream())   # the status word and outputs were made on it
        with torch.cuda.stream(stream):
            job.run()
            done = torch.cuda.Event()
            done.record(stream)
        return _InFlight(batch, job, outputs, done, now, len(batch) * output_bytes(n))

    def serve(self, requests: Iterable[Request], keep_outputs: bool = False) -> dict:
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        for r in pending:            # fit every history before the clock starts
            self.history(r.history)
        queue: List[Request] = []
        slots: List[Optional[_InFlight]] = [None] * len(self.streams)
        used = 0
        lat: List[float] = []
        intervals: List[Tuple[float, float]] = []
        cells = 0
        batches = 0
        max_overlap = 0
        results: Dict[int, Tuple[torch.Tensor, torch.Tensor]] = {}
        ids = {id(r): k for k, r in enumerate(sorted(pending, key=lambda r: r.t_arrival))}
        t0 = time.perf_counter()
        while pending or queue or any(s is not None for s in slots):
            now = time.perf_counter() - t0
            while pending and pending[0].t_arrival <= now:
                queue.append(pending.popleft())
            for k, s in enumerate(slots):        # completions
                if s is not None and s.done.query():
                    t_done = time.perf_counter() - t0
                    with torch.cuda.stream(self.streams[k]):
                        status = s.job.status.cpu()
                    if int(status.abs().sum()) != 0:
                        raise RuntimeError(f"device status {status.tolist()} in a batch of {s.batch[0].n}^3 requests")
                    for r, out in zip(s.batch, s.outputs):
                        lat.append(t_done - r.t_arrival)
                        cells += r.n ** 3
                        if keep_outputs:
                            results[ids[id(r)]] = out
                    intervals.append((s.t_launch, t_done))
                    used -= s.bytes
                    slots[k] = None
            for k in range(len(slots)):         # admissions into free slots
                if slots[k] is not None or not queue:
                    continue
                n = queue[0].n                  # the oldest request decides the grid size
                batch, extra = [], 0
                for r in queue:
                    if r.n != n:
                        continue
                    if len(batch) >= self.max_batch or used + extra + output_bytes(n) > self.budget:
                        break
                    batch.append(r)
                    extra += output_bytes(n)
                if not batch:
                    break                       # the budget is held by batches in flight
                chosen = set(map(id, batch))
                queue = [r for r in queue if id(r) not in chosen]
                slots[k] = self._launch(k, batch, time.perf_counter() - t0)
                used += extra
                batches += 1
            max_overlap = max(max_overlap, sum(s is not None for s in slots))
            if not queue and all(s is None for s in slots) and pending:
                wait = pending[0].t_arrival - (time.perf_counter() - t0)
                if wait > 2e-3:
                    time.sleep(wait - 1e-3)
        makespan = time.perf_counter() - t0
        busy = _union(intervals)
        lat.sort()

        def pct(p: float) -> float:
            return lat[min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))]

        out = {"requests": len(lat), "batches": batches, "cells": cells, "busy_s": busy, "makespan_s": makespan,
               "cells_per_s_busy": cells / busy if busy > 0 else 0.0, "slots": len(self.streams),
               "max_batches_in_flight": max_overlap,
               "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99), "mean_ms": 1e3 * sum(lat) / len(lat)}
        if keep_outputs:
            out["outputs"] = [results[k] for k in range(len(results))]
        return out


def _union(intervals: List[Tuple[float, float]]) -> float:
    """Total length covered by a set of time intervals."""
    total, end = 0.0, float("-inf")
    for a, b in sorted(intervals):
        if b <= end:
            continue
        total += b - max(a, end)
        end = b
    return total


def requests_from(schedule: Sequence[Tuple[float, int, float, Tuple[float, float, float]]]) -> List[Request]:
    return [Request(t, n, l, tuple(h)) for t, n, l, h in schedule]

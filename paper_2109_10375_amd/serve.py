"""Serving z_re requests on one GPU with continuous batching.

A request asks for the z_re field of a resident box (one per grid size) under
its own mean free path and history.  The server keeps the input fields
resident in HBM and runs a fixed number of slots, each a HIP stream with its
own workspace per grid size.  Requests arrive on the wall clock; whenever a
slot is free and the outputs fit the HBM budget, the queued requests of the
oldest request's grid size are taken as one batch and launched on that slot,
so batches keep being admitted while others are still on the device and the
work of different slots overlaps.

A batch is one box of one amber_batch_run: the forward transform of the
resident source field is shared by every requested mean free path, the rank
order of each J field by every history requested with it (Sec. 3.4.2: the
matching depends on the intensities only through their order), and requests
asking for the same (l_mfp, history) share one z_re field.  Batches of the
largest grid sizes (``exclusive_from``) fill the device on their own: they run
with no other batch in flight, so that their latency is their device time.

Completion is seen through an event per batch; a request's latency runs from
its arrival to the moment its batch is seen complete.  ``Server(..., slots=1,
max_batch=1, merge=False)`` is the plain single-box path: one request at a
time, in arrival order, each its own radiation and matching.
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


def batch_output_bytes(n: int, n_lmfp: int, n_pairs: int) -> int:
    """HBM a batch holds while it is served: one J field per distinct mean
    free path and one z_re field per distinct (l_mfp, history) pair."""
    return 4 * n ** 3 * (n_lmfp + n_pairs)


@dataclasses.dataclass
class _InFlight:
    batch: List[Request]
    job: _lib.Batch
    outputs: List[Tuple[torch.Tensor, torch.Tensor]]   # (J, z_re) of each request
    done: torch.cuda.Event
    t_launch: float
    bytes: int
    exclusive: bool


class Server:
    def __init__(self, boxes: Dict[int, Box], hbm_budget_bytes: int, max_batch: int = 16, slots: int = 2,
                 merge: bool = True, exclusive_from: Optional[int] = None):
        if slots < 1:
            raise ValueError("at least one slot")
        self.boxes = boxes
        self.budget = int(hbm_budget_bytes)
        self.max_batch = int(max_batch)
        self.merge = bool(merge)
        self.exclusive_from = max(boxes) if exclusive_from is None else int(exclusive_from)
        self.hists: Dict[Tuple[float, float, float], _lib.History] = {}
        device = next(iter(boxes.values())).S.device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]  # default priority
        self.ws: List[Dict[int, torch.Tensor]] = [dict() for _ in range(slots)]
        for n, box in boxes.items():
            if batch_output_bytes(n, 1, 1) > self.budget:
                raise ValueError(f"HBM budget {self.budget} B cannot hold one {n}^3 request")
            # two or more fields take the second spectrum: the largest workspace a box needs
            probe = _lib.BatchItem(box.plan, box.S, box.w, [1.0, 2.0], [box.S, box.S],
                                   [self.history((8.0, 4.0, 3.0))], [[box.w], [box.w]])
            need = _lib.Batch.workspace_bytes([probe])
            for k in range(slots):
                self.ws[k][n] = torch.empty(need, dtype=torch.uint8, device=device)

    def history(self, params: Tuple[float, float, float]) -> _lib.History:
        h = self.hists.get(params)
        if h is None:
            h = self.hists[params] = _lib.History.from_params(*params)
        return h

    def _plan_batch(self, batch: List[Request]):
        """Distinct mean free paths, distinct histories and the wanted pairs."""
        ls = sorted({r.l_mfp for r in batch})
        hs = sorted({r.history for r in batch})
        pairs = {(r.l_mfp, r.history) for r in batch}
        return ls, hs, pairs

    def _launch(self, slot: int, batch: List[Request], now: float) -> _InFlight:
        n = batch[0].n
        box = self.boxes[n]
        stream = self.streams[slot]
        dev = box.S.device
        ls, hs, pairs = self._plan_batch(batch)
        J = {l: torch.empty((n, n, n), dtype=torch.float32, device=dev) for l in ls}
        Z = {p: torch.empty((n, n, n), dtype=torch.float32, device=dev) for p in pairs}
        grid = [[Z.get((l, h)) for h in hs] for l in ls]
        item = _lib.BatchItem(box.plan, box.S, box.w, ls, [J[l] for l in ls], [self.history(h) for h in hs], grid)
        job = _lib.Batch([item], ws=self.ws[slot][n])
        stream.wait_stream(torch.cuda.current_stream())   # the status word and outputs were made on it
        with torch.cuda.stream(stream):
            job.run()
            done = torch.cuda.Event()
            done.record(stream)
        outputs = [(J[r.l_mfp], Z[(r.l_mfp, r.history)]) for r in batch]
        return _InFlight(batch, job, outputs, done, now, batch_output_bytes(n, len(ls), len(pairs)),
                         n >= self.exclusive_from)

    def _take(self, queue: List[Request], used: int) -> Tuple[List[Request], int]:
        """The next batch: queued requests of the oldest request's grid size,
        within the batch size and the HBM budget."""
        n = queue[0].n
        batch: List[Request] = []
        limit = self.max_batch if self.merge else 1
        for r in queue:
            if r.n != n:
                continue
            if len(batch) >= limit:
                break
            ls, _, pairs = self._plan_batch(batch + [r])
            if used + batch_output_bytes(n, len(ls), len(pairs)) > self.budget:
                break
            batch.append(r)
        if not batch:
            return batch, 0
        ls, _, pairs = self._plan_batch(batch)
        return batch, batch_output_bytes(n, len(ls), len(pairs))

    def serve(self, requests: Iterable[Request], keep_outputs: bool = False) -> dict:
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        for r in pending:            # fit every history before the clock starts
            self.history(r.history)
        queue: List[Request] = []
        slots: List[Optional[_InFlight]] = [None] * len(self.streams)
        used = 0
        lat: List[float] = []
        lat_by_n: Dict[int, List[float]] = collections.defaultdict(list)
        intervals: List[Tuple[float, float]] = []
        cells = 0
        batches = 0
        merged = 0
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
                        lat_by_n[r.n].append(t_done - r.t_arrival)
                        cells += r.n ** 3
                        if keep_outputs:
                            results[ids[id(r)]] = out
                    intervals.append((s.t_launch, t_done))
                    used -= s.bytes
                    slots[k] = None
            in_flight = [s for s in slots if s is not None]
            for k in range(len(slots)):         # admissions into free slots
                if slots[k] is not None or not queue:
                    continue
                if any(s.exclusive for s in in_flight):
                    break                       # a batch that fills the device runs alone
                exclusive = queue[0].n >= self.exclusive_from
                if exclusive and in_flight:
                    break                       # it waits for the device to drain
                batch, extra = self._take(queue, used)
                if not batch:
                    break                       # the budget is held by batches in flight
                chosen = set(map(id, batch))
                queue = [r for r in queue if id(r) not in chosen]
                slots[k] = self._launch(k, batch, time.perf_counter() - t0)
                in_flight.append(slots[k])
                used += extra
                batches += 1
                merged += len(batch) - 1
            max_overlap = max(max_overlap, sum(s is not None for s in slots))
            if not queue and all(s is None for s in slots) and pending:
                wait = pending[0].t_arrival - (time.perf_counter() - t0)
                if wait > 2e-3:
                    time.sleep(wait - 1e-3)
        makespan = time.perf_counter() - t0
        busy = _union(intervals)

        out = {"requests": len(lat), "batches": batches, "requests_merged": merged, "cells": cells, "busy_s": busy,
               "makespan_s": makespan, "cells_per_s_busy": cells / busy if busy > 0 else 0.0,
               "slots": len(self.streams), "max_batches_in_flight": max_overlap,
               "p50_ms": 1e3 * _pct(sorted(lat), 50), "p99_ms": 1e3 * _pct(sorted(lat), 99),
               "mean_ms": 1e3 * sum(lat) / len(lat),
               "p50_ms_by_n": {str(n): round(1e3 * _pct(sorted(v), 50), 3) for n, v in sorted(lat_by_n.items())},
               "p99_ms_by_n": {str(n): round(1e3 * _pct(sorted(v), 99), 3) for n, v in sorted(lat_by_n.items())}}
        if keep_outputs:
            out["outputs"] = [results[k] for k in range(len(results))]
        return out


def _pct(xs: List[float], p: float) -> float:
    return xs[min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))]


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

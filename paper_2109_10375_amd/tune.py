"""FFT schedule tuning with a persistent choice per device and grid size.

The tuner itself is amber_plan_tune (C-ABI): it times every compiled
(column pass, z pass) candidate pair of a plan on the device and keeps the
fastest.  This module remembers that choice in a JSON file keyed by the device
(architecture, compute units, memory size) and the grid size, so a later process on
the same kind of GPU sets the schedule without timing again.  An entry whose
recorded splits no longer match the library's candidate list is ignored and
replaced.  The cache path is the `cache` argument, else the environment
variable AMBER_TUNE_CACHE; with neither, the choice lives in the plan only.
"""
from __future__ import annotations

import json
import os
import tempfile
from typing import Optional

import torch

from . import _lib

CACHE_VERSION = 1


def device_key(device: Optional[torch.device] = None) -> str:
    """Identity of the GPU a schedule was timed on: architecture, compute
    units and memory size (the marketing name is left out: some tools that
    wrap a process report it empty)."""
    props = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "") or ""
    return f"{arch}|cu{props.multi_processor_count}|{props.total_memory >> 30}GiB"


def entry_key(dev_key: str, n: int) -> str:
    return f"{dev_key}|n{int(n)}"


def load(path: str) -> dict:
    """The cache's entries, or {} when the file is missing, unreadable or of
    another version."""
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    if not isinstance(data, dict) or data.get("version") != CACHE_VERSION or not isinstance(data.get("entries"), dict):
        return {}
    return data["entries"]


def store(path: str, key: str, entry: dict) -> None:
    """Adds or replaces one entry; the file is rewritten atomically."""
    entries = load(path)
    entries[key] = entry
    folder = os.path.dirname(os.path.abspath(path))
    os.makedirs(folder, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=folder, prefix=".amber_tune_", suffix=".json")
    try:
        with os.fdopen(fd, "w") as f:
            json.dump({"version": CACHE_VERSION, "entries": entries}, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.unlink(tmp)
        raise


def valid_entry(entry: dict, candidates: dict) -> bool:
    """True when the entry names candidates that exist with the same splits."""
    try:
        c, z = int(entry["col"]), int(entry["z"])
        col_split, z_split = tuple(entry["col_split"]), tuple(entry["z_split"])
    except (KeyError, TypeError, ValueError):
        return False
    if not (0 <= c < len(candidates["col"]) and 0 <= z < len(candidates["z"])):
        return False
    return tuple(candidates["col"][c]) == col_split and tuple(candidates["z"][z]) == z_split


def tune_plan(plan: _lib.Plan, S: Optional[torch.Tensor] = None, reps: int = 5, cache: Optional[str] = None) -> dict:
    """Sets plan's FFT schedule: from the cache when it holds a valid entry for
    this device and grid size, else by timing (amber_plan_tune) on S (a seeded
    uniform field when None), then recorded in the cache.  Returns the entry
    plus "cached" (whether timing was skipped)."""
    if cache is None:
        cache = os.environ.get("AMBER_TUNE_CACHE") or None
    candidates = _lib.fft_schedules(plan.n)
    key = entry_key(device_key(plan.device), plan.n)
    if cache is not None:
        entry = load(cache).get(key)
        if entry is not None and valid_entry(entry, candidates):
            plan.set_schedule(int(entry["col"]), int(entry["z"]))
            return dict(entry, cached=True)
    if S is None:
        g = torch.Generator(device=plan.device)
        g.manual_seed(plan.n)
        S = torch.rand((plan.n,) * 3, generator=g, dtype=torch.float32, device=plan.device)
    res = plan.tune(S, reps=reps)
    entry = {"col": res["col"], "z": res["z"], "col_split": list(candidates["col"][res["col"]]),
             "z_split": list(candidates["z"][res["z"]]), "ms": res["ms"], "reps": int(reps)}
    if cache is not None:
        store(cache, key, entry)
    return dict(entry, cached=False)

"""Autotuner of the batched path: bin thresholds (which kernel class a row
goes to) and the size of the persistent launches, picked by timing graph
replays of the caller's own batch.  Results are cached in a JSON file keyed by
the device and a summary of the batch.  Outputs do not depend on the choice
(the merge tree is fixed), which the tuner checks on every candidate."""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import (OPT_GRID_WAVES, OPT_GROUP_MAX, OPT_WAVE_MAX, OPT_WAVE_SMALL_MAX, Handle)

DEFAULT_CACHE = os.environ.get("BRMGPU_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "brmgpu", "autotune.json"))

KEYS = {"wave_small_max": OPT_WAVE_SMALL_MAX, "wave_max": OPT_WAVE_MAX, "group_max": OPT_GROUP_MAX,
        "grid_waves": OPT_GRID_WAVES}


def candidates():
    for ws, w, g, gw in itertools.product((32, 64), (128, 256), (512, 1024), (0, 4096, 16384, 65536)):
        yield {"wave_small_max": ws, "wave_max": w, "group_max": g, "grid_waves": gw}


def apply(h: Handle, opts: dict):
    for k, v in opts.items():
        h.set_option(KEYS[k], v)


def batch_key(triples) -> str:
    rows = sum(A.rows for A, _, _ in triples)
    nnz = sum(A.nnz for A, _, _ in triples)
    name = torch.cuda.get_device_properties(triples[0][0].rpt.device).gcnArchName
    return f"{name}|galerkin|{len(triples)}|{rows}|{nnz}"


def _time_replays(h, triples, arena, reps):
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        start.record()
        G, AP, arena = h.galerkin(triples, arena)
        end.record()
        torch.cuda.synchronize()
        times.append(start.elapsed_time(end))
    times.sort()
    return times[len(times) // 2], G, arena


def tune_galerkin(h: Handle, triples, arena=None, reps: int = 3, cache: str | None = DEFAULT_CACHE,
                  force: bool = False) -> dict:
    """Returns {"options": best, "ms": best time, "tried": n, "cached": bool}
    and leaves the best options set on the handle."""
    key = batch_key(triples)
    table = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if key in table and not force:
        apply(h, table[key]["options"])
        return {**table[key], "cached": True}
    best = None
    ref = None
    tried = 0
    for opts in candidates():
        apply(h, opts)
        G, AP, arena = h.galerkin(triples, arena)  # capture
        torch.cuda.synchronize()
        ms, G, arena = _time_replays(h, triples, arena, reps)
        tried += 1
        if ref is None:
            ref = [(g.col.clone(), g.val.clone()) for g in G]
        else:
            for (c, v), g in zip(ref, G):
                if not (torch.equal(c, g.col) and torch.equal(v.view(torch.int64), g.val.view(torch.int64))):
                    raise RuntimeError(f"output changed with options {opts}")
        if best is None or ms < best[1]:
            best = (opts, ms)
    apply(h, best[0])
    entry = {"options": best[0], "ms": best[1], "tried": tried}
    if cache:
        table[key] = entry
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return {**entry, "cached": False}

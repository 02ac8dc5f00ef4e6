"""Autotuner of the batched path: stage sizing (symbolic pass or upper-bound
slots), the wave-small kernel, bin thresholds (which kernel class a row goes
to) and the size of the persistent launches, picked by timing graph replays
of the caller's own batch.  The search is coordinate-wise: starting from the
handle's defaults, every option in turn takes each of its values with the
others at their best so far, for two passes.  Results are cached in a JSON
file keyed by the device and a summary of the batch.  Outputs do not depend
on the choice (the merge tree is fixed), which the tuner checks on every
candidate."""
from __future__ import annotations

import json
import os

import torch

from . import (OPT_BATCH_ALLOC, OPT_GRID_WAVES, OPT_GROUP_MAX, OPT_GROUP_ROWS, OPT_WAVE_MAX, OPT_WAVE_SMALL_MAX,
               Handle)

DEFAULT_CACHE = os.environ.get("BRMGPU_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "brmgpu", "autotune.json"))

KEYS = {"batch_alloc": OPT_BATCH_ALLOC, "group_rows": OPT_GROUP_ROWS, "wave_small_max": OPT_WAVE_SMALL_MAX,
        "wave_max": OPT_WAVE_MAX, "group_max": OPT_GROUP_MAX, "grid_waves": OPT_GRID_WAVES}

# the values each option may take (the first is the handle's default)
SPACE = {"batch_alloc": (0, 1), "group_rows": (1, 2, 0), "wave_small_max": (64, 32), "wave_max": (256, 128),
         "group_max": (1024, 512), "grid_waves": (0, 4096, 16384, 65536)}


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
    ref = None
    seen = {}

    def trial(opts):
        nonlocal arena, ref
        key_ = tuple(sorted(opts.items()))
        if key_ in seen:
            return seen[key_]
        apply(h, opts)
        G, AP, arena = h.galerkin(triples, arena)  # capture
        torch.cuda.synchronize()
        ms, G, arena = _time_replays(h, triples, arena, reps)
        if ref is None:
            ref = [(g.col.clone(), g.val.clone()) for g in G]
        else:
            for (c, v), g in zip(ref, G):
                if not (torch.equal(c, g.col) and torch.equal(v.view(torch.int64), g.val.view(torch.int64))):
                    raise RuntimeError(f"output changed with options {opts}")
        seen[key_] = ms
        return ms

    cur = {k: v[0] for k, v in SPACE.items()}
    best = (dict(cur), trial(cur))
    for _ in range(2):
        for k, values in SPACE.items():
            for v in values:
                cand = {**best[0], k: v}
                ms = trial(cand)
                if ms < best[1]:
                    best = (cand, ms)
    tried = len(seen)
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

"""Autotuner for the batched migration: picks the launch knobs by measurement.

The knobs are the ones the depth-stepping launch exposes (mig_tuning):
frequencies per workgroup in the two-output register-tap kernel (how many
frequency columns share a workgroup when nx is small), outputs per thread
for sections of 1025..1536 points (three: 6-8 waves per frequency, or four:
5-6 waves with more work each; the x-tile of a workgroup is always the whole
section width, so this is the tile knob), and the number of reducer
workgroups that form image rows beside the frequency workgroups.  Depth
fusion is not a knob: all depth steps of a section always run in one launch
(the plane never leaves LDS), which is the most fusion there is.  Each
candidate is timed with HIP events on the current stream; the result is
cached per batch shape for the life of the process.
"""
from __future__ import annotations

import itertools

import torch

from . import mig

_cache: dict = {}

OMEGAS_PER_GROUP = (1, 2, 4, 8)
REDUCERS = (16, 32, 48)
OUTPUTS_MID = (3, 4)


def signature(batch, desc) -> tuple:
    return (desc.ntaps, desc.nk) + tuple(
        (b["data"].shape[0], b["vel"].shape[0], b["data"].shape[1]) for b in batch)


def autotune(batch, tab32, desc, candidates=None, reps: int = 2, use_cache: bool = True):
    """Returns (best knobs, [{"tune": knobs, "ms": time}, ...])."""
    key = signature(batch, desc)
    if use_cache and key in _cache:
        return _cache[key]
    if candidates is None:
        candidates = [{"omegas_per_group": g, "reducers": r, "outputs_mid": q}
                      for g, r, q in itertools.product(OMEGAS_PER_GROUP, REDUCERS, OUTPUTS_MID)]
    need = max(mig.batch_workspace_size(batch, desc, c) for c in candidates)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=tab32.device)
    stream = torch.cuda.current_stream()
    table = []
    for c in candidates:
        mig.migrate_batched(batch, tab32, desc, tune=c, ws=ws)      # warm-up
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            mig.migrate_batched(batch, tab32, desc, tune=c, ws=ws)
        e1.record(stream)
        e1.synchronize()
        table.append({"tune": c, "ms": e0.elapsed_time(e1) / reps})
    best = min(table, key=lambda r: r["ms"])["tune"]
    _cache[key] = (best, table)
    return best, table

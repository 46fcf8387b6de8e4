"""Autotuner for launch parameters, with a JSON cache.

Candidates are timed only after they reproduce the reference candidate's
output words exactly (parity gate).  Tuned knob: the number of persistent
workgroups of an uneven-batch plan.  The cache is keyed by device
architecture, a digest of the kernel sources (a tuned choice is void once
the kernels change) and a signature of the plan (units, tiles).
"""
import json
import os

import torch

from .roofline import source_digest

_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _load():
    try:
        with open(_CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d):
    tmp = _CACHE + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, _CACHE)


def _time(fn, reps=5):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def persistent_grid(plan, candidates=None, data=None):
    """Best workgroup count for `plan` (cached).  `data`: optional list of the
    plan's device tensors, used for the parity gate (restored between runs)."""
    info = plan.info()
    key = "%s/%s/units%d/tiles%d" % (_arch(), source_digest(), info["units"], info["tiles"])
    cache = _load()
    if key in cache:
        return int(cache[key])
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    candidates = candidates or [cus, 2 * cus, 3 * cus, 4 * cus]
    best, best_ms, ref = None, None, None
    snapshot = [d.clone() for d in data] if data else None
    for g in candidates:
        plan.set_grid(g)
        if snapshot is not None:
            for d, s in zip(data, snapshot):
                d.copy_(s)
            plan.run()
            plan.status()
            out = [d.clone() for d in data]
            if ref is None:
                ref = out
            elif not all(torch.equal(x, y) for x, y in zip(out, ref)):
                continue                       # parity gate: candidate disagrees, never chosen
        ms = _time(plan.run)
        plan.status()
        if best_ms is None or ms < best_ms:
            best, best_ms = g, ms
    if snapshot is not None:
        for d, s in zip(data, snapshot):
            d.copy_(s)
    cache[key] = best
    _store(cache)
    return best

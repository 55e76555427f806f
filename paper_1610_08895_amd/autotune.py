"""Autotuner for a plan's tile side, work-item size (bin) and tile slicing.

For each candidate it builds a plan on the caller's coordinates and blocks, times a
number of batched Algorithm 1 steps (all blocks active, HIP events on the current
stream, after warm-up steps) and keeps the fastest.  Results can be cached in a JSON
file keyed by the problem's sizes and the device name, so a later run with the same
shape reuses the choice without timing.

The candidates only change how the work is partitioned; every candidate computes the
same operators (the GPU parity tests run with non-default tiles, bins and slices).
"""
import json
import os

import numpy as np
import torch

from .ops import PD, Plan, Sara

DEFAULT_CANDIDATES = (
    {"tile": 32, "bin": 1024, "slice_vis": -1},
    {"tile": 32, "bin": 512, "slice_vis": -1},
    {"tile": 16, "bin": 1024, "slice_vis": -1},
    {"tile": 32, "bin": 1024, "slice_vis": 4096},
    {"tile": 64, "bin": 1024, "slice_vis": -1},
)


def _key(n, M, d):
    """Cache key: the device's architecture and compute-unit count (marketing names differ
    between driver installs of the same part) and the problem size."""
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "").split(":")[0] or torch.cuda.get_device_name(0)
    return f"{arch}x{props.multi_processor_count}|n={n}|M={M}|d={d}"


def cached(cache, n, M, d):
    """True when the cache holds a choice for this problem size on this device."""
    if not cache or not os.path.exists(cache):
        return False
    with open(cache) as f:
        return _key(n, M, d) in json.load(f)


def time_candidate(n, uv, block_off, y_user, eps, tune, steps=10, warmup=3):
    """Mean milliseconds per batched PD step with the given tuning (all blocks active)."""
    plan = Plan(n, uv, block_off, **tune)
    yp = torch.as_tensor(np.asarray(y_user)[plan.order()], dtype=torch.complex64).to("cuda")
    sara = Sara(n)
    phin = 4.0 * n  # step sizes do not change the work of a step
    pd = PD(plan, sara, yp, eps, 0.49, 1.0 / 9.0, 1.0 / phin ** 2, 1e-3, 3.0, phin)
    for _ in range(warmup):
        pd.step()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        pd.step()
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / steps
    del pd, plan
    return ms


def tune(n, uv, block_off, y_user, eps, candidates=DEFAULT_CANDIDATES, steps=20, cache=None, log=None):
    """Returns (best tuning dict, {candidate index: ms}).  cache: JSON path or None."""
    uv = np.asarray(uv, np.float32)
    M, d = uv.shape[0], len(block_off) - 1
    key = _key(n, M, d)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f)
        if key in stored:
            return dict(stored[key]["tune"]), {}
    # two interleaved rounds, best of each candidate: a drift of the clock or of other load
    # during the sweep then does not favour whichever candidate ran at the quiet moment
    times = {}
    for rnd in range(2):
        for k, cand in enumerate(candidates):
            ms = time_candidate(n, uv, block_off, y_user, eps, cand, steps=steps)
            times[k] = min(times.get(k, ms), ms)
            if log:
                log(f"autotune {cand} (round {rnd + 1}): {ms:.4f} ms/step")
    best = dict(candidates[min(times, key=times.get)])
    if cache:
        stored = {}
        if os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f)
        stored[key] = {"tune": best, "ms": {json.dumps(candidates[k]): v for k, v in times.items()}}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(stored, f, indent=1)
    return best, times

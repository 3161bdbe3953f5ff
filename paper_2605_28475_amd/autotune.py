"""Autotuner for the apply tile shape (output states per MFMA column group, block size).

For a core and precision it times every valid shape on a seeded batch of the
requested size with HIP events on the launch stream, keeps the fastest, and
records the choice in a JSON cache keyed by (device, model, gamma, K, L,
precision, cells).  Per-cell results do not depend on the shape, so tuning only
changes speed.
"""
import json
import os

import numpy as np

from . import synth

CACHE = os.environ.get("WEFQ_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "wefq", "tune.json"))
SHAPES = [(s, b) for s in (1, 2, 4) for b in (256, 512, 768, 1024)]


def _load():
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(db):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE + ".tmp", "w") as fh:
            json.dump(db, fh, indent=1, sort_keys=True)
        os.replace(CACHE + ".tmp", CACHE)
    except OSError:
        pass


def tune(core, precision="fp32", cells=4096, reps=3, use_cache=True):
    """Choose and set the fastest tile shape; returns (slots, block, timings_ms)."""
    import torch
    from . import WefqError
    dev = torch.device("cuda", core.device)
    key = "|".join(str(x) for x in (torch.cuda.get_device_name(dev), core.model, core.gamma,
                                    core.K, core.L, precision, cells))
    db = _load() if use_cache else {}
    if key in db:
        s, b = db[key]["slots"], db[key]["block"]
        core.tune_set(precision, s, b)
        return s, b, db[key]["ms"]
    dt = torch.float64 if precision == "fp64" else torch.float32
    f = torch.tensor(synth.perturbed_maxwellian(core.K, core.L, cells, seed=synth.BASE_SEED + 97), dtype=dt, device=dev)
    q = torch.empty_like(f)
    stream = torch.cuda.current_stream(dev)
    timings = {}
    for s, b in SHAPES:
        try:
            core.tune_set(precision, s, b)
        except WefqError:
            continue                       # tile does not fit in LDS
        core.apply_Q(f, out=q, precision=precision)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, e in evs:
            a.record(stream)
            core.apply_Q(f, out=q, precision=precision)
            e.record(stream)
        torch.cuda.synchronize(dev)
        timings[f"{s},{b}"] = float(np.median([a.elapsed_time(e) for a, e in evs]))
    best = min(timings, key=timings.get)
    s, b = (int(x) for x in best.split(","))
    core.tune_set(precision, s, b)
    if use_cache:
        db[key] = {"slots": s, "block": b, "ms": timings}
        _save(db)
    return s, b, timings


def _time_plan(plan, stream, reps):
    import torch
    plan.launch(stream=stream)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, e in evs:
        a.record(stream)
        plan.launch(stream=stream)
        e.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(e) for a, e in evs]))


def tune_plan(segments, precision="fp32", blocks=(512, 768, 256), reps=3):
    """Tile shapes for a whole uneven batch, chosen by timing whole plans (graph replays), not
    segments alone: a shape that wins for a core on its own can lose inside the mix, where
    the persistent kernel's LDS size and residency are set by the largest tile and the work
    items of every core compete for the same workgroups.

    segments: list of (core, f, Q).  Coordinate descent: start from every core's default shape
    at the first block size; then, core by core in decreasing share of the plan's FLOPs, try
    every slots value with the others held, keeping the fastest; then every other block size,
    with those shapes and with the default ones (768 threads: FP32 plans of the 12-wave kernel's
    tile shapes only; other candidates that cannot be built are skipped).
    Returns (slots per segment, block, {candidate: ms}); per-cell results do not depend on it."""
    import torch
    from . import Plan, WefqError
    stream = torch.cuda.current_stream(segments[0][1].device)
    slots = [0] * len(segments)
    block = blocks[0]
    timings = {}

    def measure(sl, blk):
        key = f"block={blk} slots=" + ",".join(str(x) for x in sl)
        if key not in timings:
            try:
                plan = Plan([(c, f, q, s) for (c, f, q), s in zip(segments, sl)], precision=precision, block=blk)
            except WefqError:
                timings[key] = float("inf")        # a tile that does not fit in LDS, or a shape
                return timings[key]                # that the block size does not take
            timings[key] = _time_plan(plan, stream, reps)
            plan.close()
        return timings[key]

    best = measure(slots, block)
    order = sorted(range(len(segments)),
                   key=lambda i: -segments[i][0].info["flop_alg_per_cell"] * segments[i][1].shape[0])
    for i in order:
        for s in (1, 2, 4):
            trial = list(slots)
            trial[i] = s
            t = measure(trial, block)
            if t < best:
                best, slots = t, trial
    # every other block size, with the tuned shapes and with the default ones (the 12-wave
    # kernel of 768 threads takes only some tile shapes, which the default ones may be)
    start = list(slots)
    for blk in blocks[1:]:
        for sl in (start, [0] * len(segments)):
            t = measure(sl, blk)
            if t < best:
                best, block, slots = t, blk, list(sl)
    return slots, block, timings

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
SHAPES = [(s, b) for s in (1, 2, 4) for b in (256, 512)]


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

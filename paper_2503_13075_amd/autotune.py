"""Launch autotuner of the batched solve.

The plan's launch groups have two kinds of knobs that change speed but not
the arithmetic: the threads per workgroup of each LDS band and the LDS a
molecule may use (which moves molecules between the all-in-LDS kernel and the
partly-in-LDS ones).  ``autotune`` times the solve of a representative input
for each candidate by coordinate descent over the LDS limit and the bands,
repeated while it gains, keeps the fastest and records it in a JSON cache keyed by the device,
the plan's shape and the solve options, so that later runs on the same
workload apply it without timing again.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import _lib as L

DEFAULT_TUNING = {"band_block": [64, 128, 256, 512, 1024], "lds_limit": 0}   # a new plan's launch
BAND_CANDIDATES = [[64, 128, 256, 512, 1024]] * 3 + [[256, 512, 1024]] * 2
LDS_CANDIDATES = [0, 120 * 1024, 112 * 1024, 96 * 1024, 80 * 1024, 64 * 1024, 48 * 1024, 32 * 1024]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ilves_tuning.json")


def plan_key(plan: L.Plan, precision: int, variant: int, warm: str = "zero") -> str:
    import torch
    st = plan.stats()
    shape = [st[k] for k in ("molecules", "constraints", "atoms", "factor_entries", "updates", "sum_levels")]
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    dev = f"{getattr(props, 'gcnArchName', props.name).split(':')[0]}/{props.multi_processor_count}cu"
    text = json.dumps([dev, shape, int(precision), int(variant), warm])
    return hashlib.sha256(text.encode()).hexdigest()[:20]


def _timer(run, reps):
    """Best of two rounds of ``reps`` replays of a HIP graph capturing one
    ``run()`` (the way a tuned solve is then used: eager launches add host
    overhead that shifts the optimum), in ms per run."""
    import torch
    run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(2):
        a.record()
        for _ in range(reps):
            g.replay()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / reps)
    del g
    return best


def autotune(plan: L.Plan, run, reps: int = 10, log=None, passes: int = 3, seeds=()) -> dict:
    """Coordinate descent over the plan's tuning.  ``run()`` enqueues one
    solve on torch's current stream with the plan; it is captured in a HIP
    graph per candidate and replayed ``reps`` times (best of two rounds).
    The descent starts from the fastest of the default tuning and
    ``seeds`` (tunings found before, e.g. a recorded entry: coordinate
    descent stops in local optima, so a retune seeded with the known point
    can only keep or improve it).  A pass tries every LDS limit, then
    every block size band by band, keeping a change when it saves more than
    1%; passes repeat (the best block sizes depend on which molecules the
    LDS limit keeps in LDS, and back) until one brings no gain.  Leaves the
    plan on the fastest tuning and returns it with the default and tuned
    times (ms)."""
    cur = {"band_block": list(DEFAULT_TUNING["band_block"]), "lds_limit": DEFAULT_TUNING["lds_limit"]}
    plan.tune(**cur)
    base = best = _timer(run, reps)
    if log:
        log(f"autotune: default {cur} {base:.4f} ms")
    for sd in seeds:
        trial = {"band_block": list(sd["band_block"]), "lds_limit": int(sd["lds_limit"])}
        plan.tune(**trial)
        t = _timer(run, reps)
        if log:
            log(f"autotune: seed {trial} {t:.4f} ms")
        if t < best:
            best, cur = t, trial

    def consider(trial, what):
        nonlocal best, cur
        plan.tune(**trial)
        t = _timer(run, reps)
        if log:
            log(f"autotune: {what}: {t:.4f} ms")
        if t < best * 0.99:
            best, cur = t, trial

    for _ in range(passes):
        start = best
        for lim in LDS_CANDIDATES:
            if lim != cur["lds_limit"]:
                consider({"band_block": list(cur["band_block"]), "lds_limit": lim}, f"lds_limit {lim}")
        for band, cands in enumerate(BAND_CANDIDATES):
            for c in cands:
                if c != cur["band_block"][band]:
                    trial = {"band_block": list(cur["band_block"]), "lds_limit": cur["lds_limit"]}
                    trial["band_block"][band] = c
                    consider(trial, f"band {band} block {c}")
        if not best < start * 0.99:
            break
    plan.tune(**cur)
    return {"band_block": cur["band_block"], "lds_limit": cur["lds_limit"], "ms_default": base, "ms_tuned": best}


def load_cached(key: str, path: str = DEFAULT_CACHE):
    try:
        with open(path) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def store(key: str, tuning: dict, path: str = DEFAULT_CACHE) -> None:
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        db = {}
    db[key] = tuning
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(plan: L.Plan, run, key: str, path: str = DEFAULT_CACHE, reps: int = 10, log=None,
          store_path: str = None) -> dict:
    """Applies the cached tuning for ``key`` from ``path`` or runs
    ``autotune`` and records its result in ``store_path`` (default: the same
    file)."""
    hit = load_cached(key, path)
    if hit is not None:
        plan.tune(band_block=hit["band_block"], lds_limit=hit["lds_limit"])
        return dict(hit, cached=True)
    res = autotune(plan, run, reps=reps, log=log)
    store(key, res, store_path or path)
    return dict(res, cached=False)

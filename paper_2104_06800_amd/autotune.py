"""Autotuner of the library's launch knobs.

The knobs (voldor_knobs: local chains per block, local and coarse speculation depths, coarse
phase-A lanes per node, the order of the local level's blocks) change how a window's work is split over the chip, never its
results.  The best setting depends on the window's shape (image size, N, K, priors), so the
tuner times whole windows per (H, W, N, K, prior) bucket over a grid of settings, checks
that every setting gives the default's results bit for bit, and keeps the fastest.  Choices
are cached in a JSON file and applied to a context with `apply`.
"""
import itertools
import json
import os

import torch

SPACE = dict(local_chains=(2, 4, 8), local_spec=(1, 2, 3), coarse_spec=(4, 6, 8), coarse_lanes=(4, 8, 16),
             local_order=(1, 2))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "voldor", "knobs.json")
OUT_KEYS = ("idepth", "rigid", "pose", "conf", "stats")


def bucket(p):
    return f"{p['H']}x{p['W']}_n{p['N']}_k{p['n_candidates']}_p{int(p.get('P', 0) > 0)}"


def _timed_run(lib, p, b, pose0, reps):
    ts = []
    for r in range(reps + 1):
        b["pose"].copy_(pose0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lib.run(p, b, iters=p["iters"])
        e1.record()
        torch.cuda.synchronize()
        if r:                                   # the first run warms the caches
            ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune(lib, w, reps=3, space=None, log=None, exhaustive=False):
    """Times the window w (a synth-style dict) under knob settings of `space` and returns
    {"knobs", "ms", "default_ms", "tried"}; raises if any setting changes a result.
    exhaustive: every combination; otherwise coordinate descent (each knob in turn over its
    values, the others at their best so far)."""
    space = SPACE if space is None else space
    p = w["params"]
    b = lib.alloc(p, w["flow"], w["pose_init"], w.get("prior_idepth"), w.get("prior_pose"), w.get("prior_weight"))
    pose0 = b["pose"].clone()
    lib.set_knobs(p, None)
    default_ms = _timed_run(lib, p, b, pose0, reps)
    ref = {k: b[k].clone() for k in OUT_KEYS}
    best, best_ms, tried = {}, default_ms, 0
    names = list(space)

    def trial(knobs):
        nonlocal best, best_ms, tried
        lib.set_knobs(p, knobs)
        ms = _timed_run(lib, p, b, pose0, reps)
        for k in OUT_KEYS:
            if not torch.equal(b[k], ref[k]):
                raise RuntimeError(f"knobs {knobs} changed {k}")
        tried += 1
        if log:
            log(f"autotune {bucket(p)} {knobs}: {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = dict(knobs), ms

    if exhaustive:
        for vals in itertools.product(*(space[n] for n in names)):
            trial(dict(zip(names, vals)))
    else:
        for n in names:
            base = dict(best)
            for v in space[n]:
                trial(dict(base, **{n: v}))
    lib.set_knobs(p, best or None)
    return {"knobs": best, "ms": best_ms, "default_ms": default_ms, "tried": tried}


def load(path=DEFAULT_CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(table, path=DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def apply(lib, table, windows):
    """Sets the cached knobs of every window's bucket on the context; returns how many."""
    n = 0
    for p in windows:
        e = table.get(bucket(p))
        if e and e.get("knobs"):
            lib.set_knobs(p, e["knobs"])
            n += 1
    return n


def tune_cached(lib, windows, path=DEFAULT_CACHE, reps=3, log=None):
    """Tunes each bucket of `windows` (synth-style dicts) not yet in the cache file, saves
    the file, and applies every window's knobs."""
    table = load(path)
    for w in windows:
        key = bucket(w["params"])
        if key not in table:
            table[key] = tune(lib, w, reps=reps, log=log)
    save(table, path)
    apply(lib, table, [w["params"] for w in windows])
    return table

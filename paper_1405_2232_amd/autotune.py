"""Tile-shape autotuner for the step kernels.

Times a few candidate tile shapes (lanes per block, rows per band) of the
one-step kernel, or band heights of the two-step kernel, on a scratch copy
of the work (a lattice or a batch built by `make`, so the caller's state is
not advanced; each candidate is timed three times and its median kept)
and keeps the fastest.  Results are cached
in a JSON file keyed by the device name, the storage form and the lattice
sizes, so a later run of the same shape of work skips the timing.
"""
import hashlib
import json
import os

CANDIDATES = ((64, 4), (64, 8), (128, 4), (128, 8), (128, 16), (256, 4), (256, 8), (256, 16))
# band heights of the two-step kernel (the library's own pick is timed too)
PAIR_ROWS = (16, 24, 32, 40, 48, 64)
# single lattices also take 512-lane blocks (batches do not)
SINGLE_CANDIDATES = CANDIDATES + ((512, 4), (512, 8))
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def _key(kind, precision, sizes):
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    h = hashlib.sha1(json.dumps(sorted(sizes)).encode()).hexdigest()[:12]
    return "%s|%s|%s|%s" % (dev, kind, precision, h)


def _load():
    try:
        with open(CACHE) as fp:
            return json.load(fp)
    except (OSError, ValueError):
        return {}


def _store(cache):
    tmp = CACHE + ".tmp"
    try:
        with open(tmp, "w") as fp:
            json.dump(cache, fp, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def _time(obj, steps, treatment, repeats=3):
    """Median over `repeats` event-timed runs of `steps` steps (after two
    untimed ones): ms per step."""
    import torch
    obj.step(2, treatment)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        e0.record()
        obj.step(steps, treatment)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    return sorted(times)[repeats // 2]


def tune(make, kind, precision, sizes, treatment=1, steps=20, candidates=CANDIDATES, use_cache=True):
    """Fastest (bx, rows) for the work `make()` builds (a Lattice or Batch
    with initialised fields).  Returns ((bx, rows), {candidate: ms/step})."""
    key = _key(kind, precision, sizes)
    cache = _load() if use_cache else {}
    if key in cache:
        return tuple(cache[key]["best"]), cache[key].get("ms", {})
    obj = make()
    times = {}
    if hasattr(obj, "set_step_pairing"):
        obj.set_step_pairing(False)  # time the one-step kernel itself
    for bx, rows in candidates:
        obj.set_tiling(bx, rows)
        times["%d,%d" % (bx, rows)] = _time(obj, steps, treatment)
    del obj
    best = min(times, key=times.get)
    bx, rows = (int(v) for v in best.split(","))
    cache[key] = {"best": [bx, rows], "ms": times}
    if use_cache:
        _store(cache)
    return (bx, rows), times


def tune_pair_rows(make, kind, precision, sizes, treatment=1, steps=20, candidates=PAIR_ROWS,
                   use_cache=True):
    """Fastest band height of the two-step kernel for the work `make()`
    builds (steps even, so every launch pairs).  Returns (rows, {rows:
    ms/step}), or (0, {}) when the work does not pair steps."""
    key = _key(kind + "-pair", precision, sizes)
    cache = _load() if use_cache else {}
    if key in cache:
        return int(cache[key]["best"]), cache[key].get("ms", {})
    obj = make()
    active, own = obj.get_step_pairing()
    if not active:
        return 0, {}
    times = {}
    for rows in sorted(set(candidates) | {own}):
        obj.set_step_pairing(True, rows)
        times[str(rows)] = _time(obj, steps + (steps & 1), treatment)
    del obj
    best = int(min(times, key=times.get))
    cache[key] = {"best": best, "ms": times}
    if use_cache:
        _store(cache)
    return best, times

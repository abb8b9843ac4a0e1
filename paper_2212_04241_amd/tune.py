"""Autotuner for the layer schedule: chooses the table layout (per-slot or
slot-interleaved) and the table entries per work item (the tile, which sets
how the entries of each layer are packed into or split across workgroups)
for one junction tree, a precision and a batch size, by timing calibrations
of a representative batch of evidence cases on the device.

The best configuration depends on the tree's shape (how large the cliques
and separators of each layer are) and on the batch: small tiles give more
workgroups and more partial sums, large ones fewer of both; the interleaved
layout shares index work across the slots of a wave but runs long sums
within one lane.  Nothing here changes results beyond rounding order; the
choice is a performance decision, cached as JSON (path from the argument or
the FBN_TUNE_CACHE environment variable) under a key made of the networks'
contents, the precision, the slot count and the batch size.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import fbn

PER_SLOT, INTERLEAVED = fbn.FBN_LAYOUT_PER_SLOT, fbn.FBN_LAYOUT_INTERLEAVED

# (layout, tile entries); tile 0 is the library's default for the layout
DEFAULT_CANDIDATES = [(PER_SLOT, 0), (PER_SLOT, 512), (PER_SLOT, 2048), (PER_SLOT, 4096),
                      (INTERLEAVED, 0), (INTERLEAVED, 32), (INTERLEAVED, 128), (INTERLEAVED, 256)]


def network_key(nets, precision: int, max_slots: int, batch: int) -> str:
    """Cache key: the networks' arrays (cardinalities, parents, CPTs) and the
    run parameters."""
    h = hashlib.sha256()
    for net in (nets if isinstance(nets, (list, tuple)) else [nets]):
        for a in net.flat():
            h.update(np.ascontiguousarray(a).tobytes())
            h.update(b"|")
        h.update(b"#")
    h.update(f"p{precision}s{max_slots}b{batch}".encode())
    return h.hexdigest()


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path, data):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def measure_on_device(nets, cases, precision, max_slots, layout, tile, reps=5) -> float:
    """Milliseconds per calibration of `cases` (one per slot) with the given
    layout and tile: the median of `reps` synchronised calibrations after one
    warm-up calibration."""
    handles = [fbn.net_from_spec(n) for n in nets] if isinstance(nets, (list, tuple)) else fbn.net_from_spec(nets)
    jt = fbn.JT(handles, precision=precision, max_slots=max_slots, layout=layout, tile_entries=tile)
    slots = list(range(len(cases)))
    fbn.set_evidence_batch(jt, slots, cases)
    fbn.calibrate(jt, slots, want_results=True)          # warm-up, synchronises
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fbn.calibrate(jt, slots, want_results=True)      # synchronises
        times.append(time.perf_counter() - t0)
    jt.free()
    return 1e3 * float(np.median(times))


def tune(nets, cases, precision: int = fbn.FBN_FP32_RESCALED, max_slots: int | None = None,
         candidates=None, reps: int = 5, cache: str | None = None, measure=None, tolerance: float = 0.02) -> dict:
    """Best (layout, tile) for calibrating `cases` on the tree of `nets` (one
    network or a list, as for fbn.JT).  Returns {"layout", "tile", "ms",
    "trials": [[layout, tile, ms], ...], "cached": bool}.  A candidate replaces
    an earlier one only when faster by more than `tolerance` (a fraction), so
    that timing noise between near-equal candidates does not flip the choice
    from run to run.  `measure` replaces the device timing (same signature as
    measure_on_device)."""
    cache = cache if cache is not None else os.environ.get("FBN_TUNE_CACHE")
    max_slots = max_slots or len(cases)
    key = network_key(nets, precision, max_slots, len(cases))
    data = _load(cache)
    if key in data:
        return dict(data[key], cached=True)
    measure = measure or measure_on_device
    trials = []
    for layout, tile in (candidates or DEFAULT_CANDIDATES):
        try:
            ms = float(measure(nets, cases, precision, max_slots, layout, tile, reps))
        except fbn.FbnError:
            continue                        # e.g. a tile the tree cannot use
        trials.append([int(layout), int(tile), ms])
    if not trials:
        raise RuntimeError("no candidate configuration could be built")
    best = trials[0]
    for t in trials[1:]:
        if t[2] < best[2] * (1.0 - tolerance):
            best = t
    out = {"layout": best[0], "tile": best[1], "ms": best[2], "trials": trials}
    if cache:
        data = _load(cache)
        data[key] = out
        _store(cache, data)
    return dict(out, cached=False)

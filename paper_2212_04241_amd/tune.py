"""Autotuner for the layer schedule: chooses the table layout (per-slot or
slot-interleaved) and the table entries per work item (the tile, which sets
how the entries of each layer are packed into or split across workgroups)
for one junction tree, a precision and a batch size, by timing calibrations
of a representative batch of evidence cases on the device.  A per-slot
choice is then refined one axis at a time: the most evidence slots a layer
workgroup carries (sharing its index arithmetic) and the separator entries
per finaliser block.

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
# per-slot refinements, tried in this order, each against the best so far;
# 0 is the library's default (slots: as many as the LDS stage fits, fewer
# when the grid would not fill the chip; finaliser blocks: 4096 entries)
REFINE_AXES = (("slots_per_block", (1, 2, 4)), ("fin_block", (1024, 2048)))


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


def measure_on_device(nets, cases, precision, max_slots, layout, tile, reps=5, **knobs) -> float:
    """Milliseconds per calibration of `cases` (one per slot) with the given
    layout, tile and per-slot knobs (slots_per_block, fin_block): the median
    of `reps` synchronised calibrations after one warm-up calibration."""
    handles = [fbn.net_from_spec(n) for n in nets] if isinstance(nets, (list, tuple)) else fbn.net_from_spec(nets)
    jt = fbn.JT(handles, precision=precision, max_slots=max_slots, layout=layout, tile_entries=tile, **knobs)
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
         candidates=None, reps: int = 5, cache: str | None = None, measure=None, tolerance: float = 0.02,
         refine: bool = True) -> dict:
    """Best configuration for calibrating `cases` on the tree of `nets` (one
    network or a list, as for fbn.JT).  Returns {"layout", "tile",
    "slots_per_block", "fin_block", "ms", "trials": [[layout, tile, ms], ...],
    "refine": [[knob, value, ms], ...], "cached": bool}.  The (layout, tile)
    candidates come first; a per-slot winner is then refined along
    REFINE_AXES (when `refine`), each axis from the best so far.  A candidate
    replaces the best only when faster by more than `tolerance` (a fraction),
    so that timing noise between near-equal candidates does not flip the
    choice from run to run.  `measure` replaces the device timing (same
    signature as measure_on_device)."""
    cache = cache if cache is not None else os.environ.get("FBN_TUNE_CACHE")
    max_slots = max_slots or len(cases)
    key = network_key(nets, precision, max_slots, len(cases))
    if not refine:
        key += "-norefine"
    data = _load(cache)
    if key in data:
        return dict({"slots_per_block": 0, "fin_block": 0, "refine": []}, **data[key], cached=True)
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
    knobs = {"slots_per_block": 0, "fin_block": 0}
    ms_best, steps = best[2], []
    if refine and best[0] != INTERLEAVED:
        for name, values in REFINE_AXES:
            pick = knobs[name]
            for v in values:
                try:
                    ms = float(measure(nets, cases, precision, max_slots, best[0], best[1], reps,
                                       **dict(knobs, **{name: v})))
                except fbn.FbnError:
                    continue
                steps.append([name, int(v), ms])
                if ms < ms_best * (1.0 - tolerance):
                    ms_best, pick = ms, int(v)
            knobs[name] = pick
    out = {"layout": best[0], "tile": best[1], **knobs, "ms": ms_best, "trials": trials, "refine": steps}
    if cache:
        data = _load(cache)
        data[key] = out
        _store(cache, data)
    return dict(out, cached=False)

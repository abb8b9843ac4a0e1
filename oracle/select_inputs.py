"""Choose the accepted draw of every synthetic network and write
``fbngen/accepted.json``.  Calls only the oracle (for clique sizes) and the
seeded generator; nothing here touches the GPU library.

Acceptance rules (clique sizes are min-fill elimination cliques, in entries):
  C1  largest clique <= 4096; first attempt that meets it.
  C2  largest clique in [1e4, 1e6] (the stated range); first attempt.
  C3  largest clique in [5e6, 2e7]; up to 1000 attempts with cardinalities
      uniform on {2..63}, then attempts with P(r) proportional to 1/r.
  C4G  largest clique <= 4e6 (the memory guard proposed for the batch):
      first attempt that meets it, every drawn arc kept; up to 1000 attempts.
  C4, C5  largest clique <= 32768 (C4: the batch of small networks) and
      <= 4e6 (C5).  A few attempts by rejection, then a
      deterministic repair of attempt 0: while min-fill meets a clique above
      the cap, drop the DAG arc u->v inside that clique with the largest
      (position of v, position of u) -- or, if the clique holds no arc, the
      largest such arc touching it -- and triangulate again.

Usage:  python -m oracle.select_inputs [C1 C2 ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import fbngen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(HERE), "fbngen", "accepted.json")


def _struct_net(key, j, attempt, mode, drop=()):
    card, parents, pos = fbngen.make_structure(key, j, attempt, mode, drop, return_positions=True)
    return fbngen.Net(card, parents, []), pos


def _max_clique(net, cap):
    if oracle.probe_cap(net, cap) is not None:
        return None
    jt = oracle.compile_net(net, max_entries=cap, structure_only=True)
    return jt.max_clique, jt


def _record(jt, extra):
    d = dict(extra)
    d.update(n_cliques=jt.n_cliques, T=jt.T, K=jt.K, max_clique=jt.max_clique, H=jt.H, D=jt.D)
    return d


def select_range(key, j, lo, hi, modes, max_attempts):
    for mode in modes:
        for a in range(max_attempts):
            net, _ = _struct_net(key, j, a, mode)
            r = _max_clique(net, hi)
            if r is None:
                continue
            mx, jt = r
            if lo is None or mx >= lo:
                return _record(jt, {"attempt": a, "card_mode": mode, "drop": [], "path": "rejection"})
    raise RuntimeError(f"{key}.{j}: no attempt accepted")


def select_repair(key, j, cap, rejection_attempts):
    for a in range(rejection_attempts):
        net, _ = _struct_net(key, j, a, "uniform")
        if oracle.probe_cap(net, cap) is None:
            jt = oracle.compile_net(net, max_entries=cap, structure_only=True)
            return _record(jt, {"attempt": a, "card_mode": "uniform", "drop": [], "path": "rejection"})
    drop = []
    net, pos = _struct_net(key, j, 0, "uniform")
    while True:
        bad = oracle.probe_cap(net, cap)
        if bad is None:
            break
        inside = set(int(x) for x in bad)
        arcs = [(p, v) for v in range(net.n) for p in net.parents[v]]
        cand = [(int(pos[v]), int(pos[p]), p, v) for (p, v) in arcs if p in inside and v in inside]
        if not cand:
            cand = [(int(pos[v]), int(pos[p]), p, v) for (p, v) in arcs if p in inside or v in inside]
        _, _, p, v = max(cand)
        drop.append([int(p), int(v)])
        net, pos = _struct_net(key, j, 0, "uniform", drop)
    jt = oracle.compile_net(net, max_entries=cap, structure_only=True)
    return _record(jt, {"attempt": 0, "card_mode": "uniform", "drop": drop, "path": "repair"})


def _repair_job(args):
    key, j, cap = args
    return j, select_repair(key, j, cap, 3)


def _rejection_job(args):
    key, j, cap = args
    return j, select_range(key, j, None, cap, ["uniform"], 1000)


def main(keys):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for key in keys:
        cfg = fbngen.CONFIGS[key]
        t0 = time.time()
        res = {}
        if key in ("C4", "C4G"):
            # many independent networks: one process per core
            from multiprocessing import Pool
            job = _repair_job if key == "C4" else _rejection_job
            with Pool(max(1, min(7, (os.cpu_count() or 2) - 1))) as pool:
                for j, r in pool.imap_unordered(job, [(key, j, cfg.cap) for j in range(cfg.n_nets)]):
                    res[str(j)] = r
                    print(key, j, {k: v for k, v in r.items() if k != "drop"}, f"{time.time() - t0:.1f}s", flush=True)
            data[key] = {k: res[k] for k in sorted(res, key=int)}
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            continue
        for j in range(cfg.n_nets):
            if key == "C1":
                res[str(j)] = select_range(key, j, None, 4096, ["uniform"], 1000)
            elif key == "C2":
                res[str(j)] = select_range(key, j, 10_000, 1_000_000, ["uniform"], 1000)
            elif key == "C3":
                res[str(j)] = select_range(key, j, 5_000_000, 20_000_000, ["uniform", "inverse"], 1000)
            else:
                res[str(j)] = select_repair(key, j, cfg.cap, 3)
            print(key, j, res[str(j)] if key != "C4" else {k: v for k, v in res[str(j)].items() if k != "drop"},
                  f"{time.time() - t0:.1f}s", flush=True)
        data[key] = res
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["C1", "C2", "C3", "C4", "C5"])

#!/usr/bin/env python3
"""Evidence queries/s and table-op HBM bandwidth of junction-tree inference on
one MI355X: the FP32 path with rescaled separators, all cases of the workload
batched into one calibration, against the plain FP64 path run one query at a
time, with the FP64 oracle timed on the host cores beside them.

A step is one calibration (collect + distribute + posteriors, every layer
kernel) of every evidence case of the workload, with the network and the
evidence already resident in device memory; posteriors stay on the device.

With --workload C4 the 256 networks form one forest junction tree and a
step calibrates 64 slots, each holding one case of every network (16384
queries).  With --workload C5 eight trees stay resident and serve a Poisson
trace of queries with continuous batching; a step is one closed-loop replay
of the trace, and latency percentiles come with it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload C2|C4|C5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
PROFILES = os.path.join(ROOT, "profiles")
# the sources a kernel's byte counters depend on: counters taken before a
# change to any of them no longer describe the kernel
KERNEL_SOURCES = ["paper_2212_04241_amd/csrc/kernels.hip", "paper_2212_04241_amd/csrc/kernels_interleaved.hip",
                  "paper_2212_04241_amd/csrc/kernels.h", "paper_2212_04241_amd/csrc/api.cpp",
                  "paper_2212_04241_amd/csrc/plan.cpp", "paper_2212_04241_amd/csrc/plan.h",
                  "paper_2212_04241_amd/csrc/fbn_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha256():
    """Hash of the kernel sources' code: comments and blank lines removed, so
    that only a change to the code itself invalidates recorded counters."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            for line in fh:
                line = re.sub(r"//.*$", "", line).rstrip()
                if line:
                    h.update(line.encode() + b"\n")
    return h.hexdigest()


# kernel behind each timed launch kind, per-slot and slot-interleaved layouts
KIND_KERNEL = {"collect": "k_collect", "collect_finalise": "k_fin_collect", "distribute": "k_dist_gather",
               "distribute_finalise": "k_fin_distribute", "posteriors": "k_marginals"}
KIND_KERNEL_IL = {"collect": "k_collect_i", "collect_finalise": "k_fin_collect_i", "distribute": "k_dist_i",
                  "distribute_finalise": "k_fin_distribute_i", "posteriors": "k_marginals_i"}


def counted_traffic(workload, kernel, layout, tile, tiles=None, slots=None):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary (copy-scaled), or None when there is no
    summary for this workload and kernel, it was taken with another layout,
    tile or slot count, or the kernel sources changed since the counters were
    taken."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != sources_sha256():
        return None
    if kv.get("layout") != str(int(layout)) or kv.get("tile") != str(int(tile)):
        return None
    if "tiles" in kv and (tiles is None or kv["tiles"] != ",".join(str(int(t)) for t in tiles)):
        return None
    if "slots" in kv and (slots is None or kv["slots"] != str(int(slots))):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline_of(prof, workload, layout, tile, note=None, interleaved=False, tiles=None, slots=None):
    """Roofline object for the kernel kind with the most time in `prof`
    (kind -> (ms, launches, algorithmic bytes)), measured by HIP events."""
    kind = max(prof, key=lambda k: prof[k][0])
    ms, launches, byts = prof[kind]
    achieved = byts / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    kernel = (KIND_KERNEL_IL if interleaved else KIND_KERNEL)[kind]
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counted_traffic(workload, kernel, layout, tile, tiles, slots),
         "kernel": f"{kernel}<float>", "launches": launches,
         "avg_launch_us": round(1e3 * ms / max(launches, 1), 3),
         "bytes_per_launch": byts / max(launches, 1),
         "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)"}
    if note:
        r["measured_on"] = note
    return r


class Workload:
    """The networks and evidence of one preset.  A slot is one evidence case
    of the junction tree; with several networks (C4) the tree is a forest of
    all of them and one slot carries one case of every network, so a slot
    answers len(nets) queries."""

    def __init__(self, key, n_cases=None):
        import fbngen
        self.key = key
        cfg = fbngen.CONFIGS[key]
        if key in ("C4", "C4G"):
            self.nets = [fbngen.make_net(key, j) for j in range(cfg.n_nets)]
            self.cases = [fbngen.make_cases(key, n, j) for j, n in enumerate(self.nets)]
            off = fbngen.forest_offsets(self.nets)
            self.slot_cases = [fbngen.forest_case(off, self.cases, s) for s in range(cfg.n_cases)]
        else:
            self.nets = [fbngen.make_net(key, 0)]
            self.cases = [fbngen.make_cases(key, self.nets[0])]
            if n_cases:
                self.cases[0] = self.cases[0][:n_cases]
            self.slot_cases = self.cases[0]
        self.per_slot = len(self.nets)
        self.marg_off = np.concatenate([[0], np.cumsum([int(np.sum(n.card)) for n in self.nets])]).astype(int)
        self.marg = int(self.marg_off[-1])

    def handles(self, fbn):
        h = [fbn.net_from_spec(n) for n in self.nets]
        return h if len(h) > 1 else h[0]

    def sample(self, k):
        """(network, case index) pairs of the accuracy and host samples."""
        if len(self.nets) == 1:
            return [(0, i) for i in range(min(k, len(self.cases[0])))]
        per = max(1, k // 8)
        return [(j, i) for j in range(min(8, len(self.nets))) for i in range(min(per, len(self.cases[j])))]


def workload_config(key, W, jt_stats, n_slots):
    import fbngen
    return {
        "workload": f"{key}: {fbngen.CONFIGS[key].description}",
        "queries_per_step": n_slots * W.per_slot,
        "networks": len(W.nets),
        "slots": n_slots,
        "variables": jt_stats["n_vars"],
        "cliques": jt_stats["n_cliques"],
        "table_entries_T": jt_stats["T"],
        "max_clique_entries": jt_stats["max_clique"],
        "separator_entries": jt_stats["sep_total"],
        "layers_collect": jt_stats["H"] + 1,
        "layers_distribute": jt_stats["D"] + 1,
    }


def copy_gbps(mib=1024, reps=5):
    """Achievable HBM bandwidth of a plain device-to-device copy (read +
    write bytes over the median copy time), the ceiling shown beside the
    peak."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * (mib << 20) / float(np.median(times)) / 1e9


def fitting_slots(fbn, W, precision, layout, tile, frac=0.9):
    """How many of the workload's slots a device build of this precision and
    layout can hold in `frac` of the free device memory (host-only build
    for the footprint)."""
    import torch
    n = len(W.slot_cases)
    jt = fbn.JT(W.handles(fbn), precision=precision, max_slots=n, layout=layout, tile_entries=tile, host_only=True)
    st = jt.stats
    fixed = st["device_bytes"] - n * st["slot_bytes"]
    free, _ = torch.cuda.mem_get_info()
    return max(1, min(n, int((frac * free - fixed) // max(1, st["slot_bytes"]))))


def time_batched(fbn, W, precision, steps, warmup, profile, layout=0, tile=0, event_every=1, n_cases=None):
    """Time `steps` calibrations of the whole batch.  With profile, one
    untimed warm-up step times every kernel kind (the per-kind breakdown
    returned as `kinds`), and timed steps record HIP events around the
    launches of the kind with the most time only, in one step of every
    `event_every` (each event pair is a marker on the stream that costs a
    few microseconds, so the other steps run without them)."""
    import torch
    cases = W.slot_cases[:n_cases] if n_cases else W.slot_cases
    n = len(cases)
    # the layer sequence replayed as one captured graph (steps that record
    # kernel events run it eagerly)
    stream = torch.cuda.Stream()
    handles = W.handles(fbn)
    t0 = time.perf_counter()
    jt = fbn.JT(handles, precision=precision, max_slots=n, layout=layout, tile_entries=tile,
                stream=stream.cuda_stream)
    stream.synchronize()
    jt._build_s = time.perf_counter() - t0  # compile, plan, device allocation and upload
    fbn.set_graph_mode(jt, True)
    jt._bench_stream = stream           # keeps the stream alive as long as the tree
    slots = list(range(n))
    fbn.set_evidence_batch(jt, slots, cases)
    for _ in range(max(warmup, 1)):
        fbn.calibrate(jt, slots)
    kinds = None
    if profile:
        fbn.jt_profile_read(jt)
        fbn.jt_profile_enable(jt, True)
        fbn.calibrate(jt, slots)
        kinds = fbn.jt_profile_read(jt)
        dominant = max(kinds, key=lambda k: kinds[k][0])
        fbn.jt_profile_kinds(jt, [dominant])
    fbn.jt_profile_read(jt)             # synchronises; clears counters
    t0 = time.perf_counter()
    for i in range(steps):
        if profile:
            fbn.jt_profile_enable(jt, (i + 1) % event_every == 0 or (i == steps - 1 and steps < event_every))
        fbn.calibrate(jt, slots)
    prof = fbn.jt_profile_read(jt)      # synchronises the stream
    dt = time.perf_counter() - t0
    fbn.jt_profile_enable(jt, False)
    fbn.jt_profile_kinds(jt, None)
    post, lp, st = fbn.query_all(jt, slots, W.marg)
    if profile:
        prof = {k: v for k, v in prof.items() if v[1] > 0}
    return jt, dt, (prof, kinds), post, lp, st


def time_plain(fbn, W, n_queries, graph=True, precision=None):
    """One query per calibration on the query's own network, waiting for
    each result (a per-query engine); with graph, the layer sequence is
    replayed as one captured graph.  Returns q/s, latencies and, per
    network used, (case indices, post, log_pe, status)."""
    import torch
    groups = {}
    for j, i in W.sample(n_queries):
        groups.setdefault(j, []).append(i)
    stream = torch.cuda.Stream()
    lat, res, dt = [], {}, 0.0
    for j, idx in groups.items():
        net = W.nets[j]
        jt = fbn.JT(fbn.net_from_spec(net), precision=fbn.FBN_FP64 if precision is None else precision,
                    max_slots=len(idx), stream=stream.cuda_stream)
        if graph:
            fbn.set_graph_mode(jt, True)
        slots = list(range(len(idx)))
        fbn.set_evidence_batch(jt, slots, [W.cases[j][i] for i in idx])
        for s in slots[:3]:             # warm-up (uploads evidence)
            fbn.calibrate(jt, [s], want_results=True)
        t0 = time.perf_counter()
        for s in slots:
            a = time.perf_counter()
            fbn.calibrate(jt, [s], want_results=True)
            lat.append(time.perf_counter() - a)
        dt += time.perf_counter() - t0
        post, lp, st = fbn.query_all(jt, slots, int(np.sum(net.card)))
        res[j] = (idx, post, lp, st)
        jt.free()
    return len(lat) / dt, np.array(lat), res


def time_with_host_io(fbn, W, precision, steps, layout=0, tile=0):
    """Same batch, counting evidence upload and posterior download (PCIe)."""
    cases = W.slot_cases
    n = len(cases)
    jt = fbn.JT(W.handles(fbn), precision=precision, max_slots=n, layout=layout, tile_entries=tile)
    slots = list(range(n))
    marg = W.marg
    fbn.set_evidence_batch(jt, slots, cases)
    fbn.calibrate(jt, slots)
    fbn.query_all(jt, slots, marg)
    t0 = time.perf_counter()
    for _ in range(steps):
        fbn.set_evidence_batch(jt, slots, cases)
        fbn.calibrate(jt, slots)
        fbn.query_all(jt, slots, marg)
    return n * W.per_slot * steps / (time.perf_counter() - t0)


def oracle_one_core(ojts, pairs, cases_of, limit_s=10.0):
    """The oracle on one host core: median seconds per query over `pairs`
    ((network, case) keys), run one after another, stopping after limit_s."""
    times = []
    t_end = time.perf_counter() + limit_s
    for j, i in pairs:
        a = time.perf_counter()
        ojts[j].query(*cases_of(j, i))
        times.append(time.perf_counter() - a)
        if time.perf_counter() > t_end:
            break
    med = float(np.median(times))
    return {"median_ms_per_query": round(1e3 * med, 3), "queries_per_s_one_core": round(1.0 / med, 2),
            "queries_timed": len(times)}


def host_cpu() -> dict:
    """The host the CPU baseline ran on: logical cores and the model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(W, seconds):
    import oracle
    sample = W.sample(200 if len(W.nets) == 1 else 512)
    ojts = {j: oracle.compile_net(W.nets[j]) for j in sorted({j for j, _ in sample})}
    threads = max(1, min(16, os.cpu_count() or 1))
    done = 0
    t0 = time.perf_counter()

    def run(k):
        j, i = sample[k % len(sample)]
        ojts[j].query(*W.cases[j][i])
        return 1

    with ThreadPoolExecutor(threads) as ex:
        while time.perf_counter() - t0 < seconds:
            done += sum(ex.map(run, range(done, done + 4 * threads)))
    dt = time.perf_counter() - t0
    what = (f"the first {len(sample)} cases" if len(W.nets) == 1 else
            f"{len(sample)} (network, case) queries: the first {len(sample) // len(ojts)} cases of the first "
            f"{len(ojts)} networks")
    return {"value": done / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} oracle queries cycling over {what}, {dt:.1f} s, "
                      f"{threads} threads (one query per thread at a time)", "host": host_cpu()}, ojts


def accuracy(W, ojts, get, pairs, fp32):
    """get(j, i) -> (posterior slice of network j, case i; its log P(e) or
    None where the path only reports a sum over networks)."""
    import oracle
    worst_abs = worst_rel = worst_lp = 0.0
    for j, i in pairs:
        if j not in ojts:
            ojts[j] = oracle.compile_net(W.nets[j])
        olp, op = ojts[j].query(*W.cases[j][i])
        post, lp = get(j, i)
        err = np.abs(post - op)
        worst_abs = max(worst_abs, float(err.max()))
        worst_rel = max(worst_rel, float(np.max(err / np.maximum(np.abs(op), 1e-300))))
        if lp is not None:
            worst_lp = max(worst_lp, abs(float(lp) - olp))
    return {"queries_checked": len(pairs), "max_abs_err": worst_abs,
            "max_rel_err": None if fp32 else worst_rel, "max_logpe_err": worst_lp}


def forest_logpe_err(W, ojts, lp, slot):
    """|log P(e) of a forest slot - sum over networks of the oracle's|."""
    import oracle
    tot = 0.0
    for j in range(len(W.nets)):
        if j not in ojts:
            ojts[j] = oracle.compile_net(W.nets[j])
        tot += ojts[j].query(*W.cases[j][slot])[0]
    return abs(float(lp[slot]) - tot)


def profile_full_batches(fbn, srv, queries):
    """Per kernel kind (ms, launches, algorithmic bytes) over one eager, HIP-
    event-timed calibration of a full batch (the first trace queries of its
    network) on every resident tree."""
    prof = {}
    for k, jt in enumerate(srv.jts):
        qs = [q for q in queries if q.net == k][: srv.slots]
        if not qs:
            continue
        sl = list(range(len(qs)))
        fbn.set_evidence_batch(jt, sl, [(q.vars, q.states) for q in qs])
        fbn.jt_profile_read(jt)
        fbn.jt_profile_enable(jt, True)
        fbn.calibrate(jt, sl)
        for kind, (ms, launches, byts) in fbn.jt_profile_read(jt).items():
            a = prof.setdefault(kind, [0.0, 0, 0.0])
            a[0] += ms
            a[1] += launches
            a[2] += byts
        fbn.jt_profile_enable(jt, False)
    return prof


def copy_calibration():
    """A plain device copy of known size, so that byte counters taken in the
    same run can be scaled (read 512 MiB, write 512 MiB, three times)."""
    import torch
    src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("[bench] copy calibration: 3 x 512 MiB device copies")


def bench_served(args, fbn):
    """The served workload: eight resident networks, a Poisson trace of
    evidence queries, continuous batching with footprint admission (FP32),
    against the plain per-query FP64 engine on the same trace.  Load points:
    closed loop (every query available at once) for both; open loop at 0.8 x
    the plain engine's saturation rate for both; open loop at 0.8 x the
    served saturation rate for the served path."""
    import fbngen
    from paper_2212_04241_amd.serve import Server, serve_plain, trace_queries
    nets = [fbngen.make_net("C5", j) for j in range(8)]
    times, which, fracs, seeds = fbngen.make_arrivals("C5")
    n = min(args.trace, len(times))
    cases = [fbngen.case_for_arrival(nets[int(which[i])], float(fracs[i]), int(seeds[i])) for i in range(n)]
    queries = trace_queries(times[:n], which[:n], cases)
    log(f"[bench] C5: 8 networks, {n} trace queries")
    t0 = time.perf_counter()
    # tile per tree: --tiles, else --tile for all, else the tuner's pick for a
    # full batch of each tree
    if args.tiles and args.tiles != "auto":
        tl = [int(x) for x in args.tiles.split(",")]
        tiles = tl * len(nets) if len(tl) == 1 else tl
    else:
        tiles = args.tile or None
    srv = Server(nets, budget_bytes=int(args.budget_gb * (1 << 30)), max_batch=args.max_batch,
                 tile=tiles, layout=args.layout, warm=not args.kernels_only)
    server_s = time.perf_counter() - t0
    log(f"[bench] server up in {server_s:.1f} s: {srv.slots} slots per tree, "
        f"{srv.device_bytes / 2**30:.2f} GiB resident, plan {srv.planned_bytes / 2**30:.2f} GiB of "
        f"{args.budget_gb} GiB, tiles {srv.tiles}")
    if args.kernels_only:
        prof = profile_full_batches(fbn, srv, queries)
        srv.close()
        if args.copy_calibration:
            copy_calibration()
        roofline = roofline_of({k: tuple(v) for k, v in prof.items()}, "C5", args.layout, args.tile,
                               "one full batch per resident tree, eager launches, HIP events",
                               interleaved=args.layout == 2, tiles=srv.tiles, slots=srv.slots)
        print(json.dumps({"workload": "C5", "tiles": srv.tiles, "roofline": roofline,
                          "kernel_ms_one_batch_per_tree": {k: v[0] for k, v in prof.items()},
                          "kernel_launches": {k: v[1] for k, v in prof.items()}}), flush=True)
        return
    keep = list(range(min(200, n)))
    for _ in range(args.warmup):
        srv.run(queries[: min(n, 256)])
    # (i) closed loop, served: `steps` replays of the trace
    tot_q = tot_t = 0.0
    sat = None
    for _ in range(args.steps):
        r = srv.run(queries, None, keep=keep if sat is None else None)
        sat = sat or r
        tot_q += n
        tot_t += r.wall
    qps_served = tot_q / tot_t
    log(f"[bench] served closed loop: {qps_served:.1f} q/s ({args.steps} x {n} queries), "
        f"p50 {1e3 * sat.percentile(50):.2f} ms")
    # useful bandwidth: the materialised-Hugin table bytes (3 T w) of each
    # query's own network, per second
    T_net = [int(jt.stats["T"]) for jt in srv.jts]
    bytes_per_query = float(np.mean([3.0 * T_net[q.net] for q in queries]))
    # dominant kernel: one profiled (eager) full batch per tree
    prof = profile_full_batches(fbn, srv, queries)
    # plain FP64 engine, closed loop over a prefix
    plain_sat = serve_plain(nets, queries, None, limit=args.plain_queries, keep=keep)
    log(f"[bench] plain fp64 closed loop: {plain_sat.qps:.1f} q/s over {len(plain_sat.latency)} queries")
    # (ii) open loop at 0.8 x plain saturation, both paths
    lam2 = 0.8 * plain_sat.qps
    srv_2 = srv.run(queries, lam2)
    plain_2 = serve_plain(nets, queries, lam2, limit=args.plain_queries)
    # (iii) open loop at 0.8 x served saturation
    lam3 = 0.8 * qps_served
    srv_3 = srv.run(queries, lam3)
    log(f"[bench] open loop {lam2:.0f}/s: served p50 {1e3 * srv_2.percentile(50):.2f} ms p99 "
        f"{1e3 * srv_2.percentile(99):.2f}; plain p50 {1e3 * plain_2.percentile(50):.2f} p99 "
        f"{1e3 * plain_2.percentile(99):.2f}; open loop {lam3:.0f}/s: served p50 {1e3 * srv_3.percentile(50):.2f} "
        f"p99 {1e3 * srv_3.percentile(99):.2f}")
    slots, resident, srv_tiles = srv.slots, srv.device_bytes, list(srv.tiles)
    status_nonzero = int(np.count_nonzero(sat.status)) + int(np.count_nonzero(plain_sat.status))
    fallbacks = int(np.count_nonzero(sat.precision == fbn.FBN_FP64))
    srv.close()
    # the same server with the shrinking reduction (only evidence-consistent
    # entries read and written), one closed-loop replay: what it changes
    shrink = None
    if not args.no_shrink_compare:
        srv_s = Server(nets, budget_bytes=int(args.budget_gb * (1 << 30)), max_batch=args.max_batch,
                       tile=srv_tiles, layout=args.layout, shrink_evidence=True)
        srv_s.run(queries[: min(n, 256)])
        rs = srv_s.run(queries, None, keep=keep)
        sprof = profile_full_batches(fbn, srv_s, queries)
        same = all(np.array_equal(rs.post[i], sat.post[i]) and rs.log_pe[i] == sat.log_pe[i] for i in keep)
        srv_s.close()
        dk = max(prof, key=lambda k: prof[k][0])
        shrink = {"queries_per_s": round(rs.qps, 1), "p50_ms": round(1e3 * rs.percentile(50), 3),
                  "results_bitwise_equal_on_first": len(keep) if same else -1,
                  "speedup_vs_streaming_every_entry": round(rs.qps / max(qps_served, 1e-9), 3),
                  "table_bytes_streamed_vs_every_entry": round(
                      sum(v[2] for k, v in sprof.items() if k in ("collect", "distribute")) /
                      max(sum(v[2] for k, v in prof.items() if k in ("collect", "distribute")), 1.0), 3),
                  f"{dk}_ms_one_batch_per_tree": round(sprof[dk][0], 3)}
        log(f"[bench] served with the shrinking reduction: {rs.qps:.1f} q/s "
            f"(x{shrink['speedup_vs_streaming_every_entry']}, bytes x{shrink['table_bytes_streamed_vs_every_entry']})")

    roofline = roofline_of({k: tuple(v) for k, v in prof.items()}, "C5", args.layout, args.tile,
                           "one full batch per resident tree, eager launches, HIP events",
                           interleaved=args.layout == 2, tiles=srv_tiles, slots=slots)
    roofline["stream_copy_GBps"] = round(copy_gbps(), 1)

    def lat(r):
        return {"queries_per_s": round(r.qps, 1), "p50_ms": round(1e3 * r.percentile(50), 3),
                "p99_ms": round(1e3 * r.percentile(99), 3), "queries": int(len(r.latency))}

    out = {
        "metric": "evidence queries/sec and table-op HBM GB/s, FP32-served vs plain FP64, 1 GPU",
        "value": round(qps_served, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * tot_t / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "setup_ms": {"server_compile_build_upload_warm": round(1e3 * server_s, 3)},
        "config": {"workload": f"C5: {fbngen.CONFIGS['C5'].description}", "networks": 8,
                   "trace_queries": n, "budget_GiB": args.budget_gb, "slots_per_tree": slots,
                   "resident_GiB": round(resident / 2**30, 3), "max_batch": args.max_batch,
                   "layout": "interleaved" if args.layout == 2 else "per-slot", "tile_per_tree": srv_tiles,
                   "step": "one closed-loop replay of the trace"},
        "roofline": roofline,
        "paths": {
            "served_fp32_closed_loop": lat(sat) | {"batches": sat.batches, "fp64_fallbacks": fallbacks,
                                                   "useful_GBps": round(qps_served * bytes_per_query * 4 / 1e9, 1),
                                                   "kernel_ms_one_batch_per_tree":
                                                       {k: round(v[0], 3) for k, v in prof.items()}},
            "plain_fp64_closed_loop": lat(plain_sat) | {
                "useful_GBps": round(plain_sat.qps * bytes_per_query * 8 / 1e9, 1)},
            "open_loop_at_0.8x_plain": {"rate_per_s": round(lam2, 1), "served": lat(srv_2), "plain": lat(plain_2)},
            "open_loop_at_0.8x_served": {"rate_per_s": round(lam3, 1), "served": lat(srv_3),
                                         "plain": "unstable at this rate (above its saturation)"},
            "served_vs_plain": round(qps_served / max(plain_sat.qps, 1e-9), 2),
            "served_fp32_shrinking_reduction_closed_loop": shrink,
        },
        "status_nonzero": status_nonzero,
    }
    if not args.no_cpu_baseline:
        # the oracle's leg: the CPU baseline and the accuracy check
        import oracle
        sample = keep
        threads = max(1, min(16, os.cpu_count() or 1))
        t1 = time.perf_counter()
        used = sorted({queries[i].net for i in sample})
        with ThreadPoolExecutor(len(used)) as ex:
            ojts = dict(zip(used, ex.map(lambda k: oracle.compile_net(nets[k]), used)))
        log(f"[bench] oracle compiled in {time.perf_counter() - t1:.1f} s")
        done = 0
        results = {}
        t0 = time.perf_counter()

        def run(k):
            i = sample[k % len(sample)]
            q = queries[i]
            lp, post = ojts[q.net].query(q.vars, q.states)
            if k < len(sample):
                results[i] = (lp, post)
            return 1

        with ThreadPoolExecutor(threads) as ex:
            while time.perf_counter() - t0 < args.cpu_seconds:
                done += sum(ex.map(run, range(done, done + threads)))
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
                               "sample": f"{done} oracle queries over the first {len(sample)} trace queries, "
                                         f"{dt:.1f} s, {threads} threads (one query per thread at a time)",
                               "host": host_cpu()}
        out["cpu_baseline"]["one_core"] = oracle_one_core(
            ojts, [(queries[i].net, i) for i in sample], lambda j, i: (queries[i].vars, queries[i].states))
        e32 = e64 = l32 = l64 = 0.0
        for i, (olp, op) in results.items():
            e32 = max(e32, float(np.max(np.abs(sat.post[i] - op))))
            e64 = max(e64, float(np.max(np.abs(plain_sat.post[i] - op))))
            l32 = max(l32, abs(sat.log_pe[i] - olp))
            l64 = max(l64, abs(plain_sat.log_pe[i] - olp))
        out["accuracy"] = {"queries_checked": len(results),
                           "served_fp32": {"max_abs_err": e32, "max_logpe_err": l32},
                           "plain_fp64": {"max_abs_err": e64, "max_logpe_err": l64}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C5",
                    help="C5 (default: the served comparison the metric names), C1, C2, C3 or C4")
    ap.add_argument("--plain-queries", type=int, default=300)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true", help="time only the FP32 batched path (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain 512 MiB device copies (reference for byte counters)")
    ap.add_argument("--layout", type=int, default=0, help="table layout: 0 auto, 1 per slot, 2 interleaved")
    ap.add_argument("--tile", type=int, default=0, help="table entries per work item (0: the library default)")
    ap.add_argument("--event-every", type=int, default=4,
                    help="HIP events around the dominant kernel in one timed step of every N")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (layout and tile from --layout / --tile)")
    ap.add_argument("--cases", type=int, default=0, help="single-network workloads: the first N cases only")
    ap.add_argument("--trace", type=int, default=4096, help="C5: trace queries")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="C5: device-memory budget, GiB")
    ap.add_argument("--max-batch", type=int, default=64, help="C5: slots per resident tree at most")
    ap.add_argument("--tiles", default="2048",
                    help="C5: tile per tree, one value for all or comma-separated per tree; 'auto' times "
                         "the candidates on the device (it picks 2048 for all or all but one of the trees)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="C5: only the profiled full batch per resident tree (for counter runs)")
    ap.add_argument("--no-shrink-compare", action="store_true",
                    help="C5: skip the closed-loop replay with the shrinking reduction")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; sharding the path across "
                                   "GPUs is not built", "n_gpus": args.gpus}))
        sys.exit(2)

    from paper_2212_04241_amd import fbn

    key = args.workload
    if key == "C5":
        return bench_served(args, fbn)
    W = Workload(key, args.cases or None)
    n = len(W.slot_cases)
    q = n * W.per_slot
    log(f"[bench] {key}: {len(W.nets)} network(s), {sum(x.n for x in W.nets)} variables, {n} slots, "
        f"{q} queries per step")

    # layout and tile: the autotuner's measured choice for this batch (before
    # the timed region), unless fixed on the command line
    tuned = None
    if not args.no_tune and not args.layout and not args.tile:
        from paper_2212_04241_amd import tune
        nets = W.nets if len(W.nets) > 1 else W.nets[0]
        t0 = time.perf_counter()
        tuned = tune.tune(nets, W.slot_cases, fbn.FBN_FP32_RESCALED)
        args.layout, args.tile = tuned["layout"], tuned["tile"]
        log(f"[bench] tuned in {time.perf_counter() - t0:.1f} s: layout {args.layout}, tile {args.tile} "
            f"({tuned['ms']:.3f} ms per calibration)")
    # junction-tree compile alone (host: triangulation, tree, layouts, maps,
    # plan), timed apart from the device build and upload
    t0 = time.perf_counter()
    fbn.JT(W.handles(fbn), precision=fbn.FBN_FP32_RESCALED, max_slots=n, layout=args.layout,
           tile_entries=args.tile, host_only=True).free()
    compile_s = time.perf_counter() - t0
    # FP32 batched (the headline path), kernel timing by HIP events
    jt32, dt32, (prof32, kinds32), post32, lp32, st32 = time_batched(fbn, W, fbn.FBN_FP32_RESCALED, args.steps,
                                                                     args.warmup, True, args.layout, args.tile,
                                                                     args.event_every)
    stats = jt32.stats
    build_s = jt32._build_s
    qps32 = q * args.steps / dt32
    log(f"[bench] fp32 batched: {qps32:.1f} q/s, {1e3 * dt32 / args.steps:.3f} ms/step")
    jt32.free()
    if args.copy_calibration:
        copy_calibration()
    roofline = roofline_of(prof32, key, args.layout, args.tile, interleaved=bool(stats["interleaved"]))
    if not args.fp32_only:
        roofline["stream_copy_GBps"] = round(copy_gbps(), 1)
    if args.fp32_only:
        # profiling runs: the headline path alone
        print(json.dumps({"value": round(qps32, 1), "unit": "queries/s", "ms_per_step": 1e3 * dt32 / args.steps,
                          "roofline": roofline,
                          "kernel_ms_one_profiled_step": {k: v[0] for k, v in kinds32.items()},
                          "kernel_launches_one_step": {k: v[1] for k, v in kinds32.items()}}), flush=True)
        return
    # FP64 batched
    steps64 = max(1, args.steps // 2)
    # float64 tables take twice the memory: as many cases as fit
    n64 = fitting_slots(fbn, W, fbn.FBN_FP64, args.layout, args.tile)
    jt64, dt64, _, post64, lp64, st64 = time_batched(fbn, W, fbn.FBN_FP64, steps64, 1, False, args.layout,
                                                     args.tile, n_cases=n64)
    qps64b = n64 * W.per_slot * steps64 / dt64
    jt64.free()
    log(f"[bench] fp64 batched: {qps64b:.1f} q/s ({n64} slots)")
    # FP64 plain, one query per calibration
    qps_plain, lat, plain = time_plain(fbn, W, args.plain_queries)
    log(f"[bench] fp64 plain (graph replay): {qps_plain:.1f} q/s, p50 {1e3 * np.median(lat):.3f} ms")
    qps_plain_eager, lat_e, _ = time_plain(fbn, W, args.plain_queries, graph=False)
    log(f"[bench] fp64 plain (eager launches): {qps_plain_eager:.1f} q/s")
    qps_plain32, lat32, _ = time_plain(fbn, W, args.plain_queries, precision=fbn.FBN_FP32_RESCALED)
    log(f"[bench] fp32 plain (graph replay): {qps_plain32:.1f} q/s, p50 {1e3 * np.median(lat32):.3f} ms")
    qps_io = time_with_host_io(fbn, W, fbn.FBN_FP32_RESCALED, max(1, args.steps // 4), args.layout, args.tile)
    log(f"[bench] fp32 batched with host i/o: {qps_io:.1f} q/s")


    T = stats["T"]
    out = {
        "metric": "evidence queries/sec and table-op HBM GB/s, FP32-served vs plain FP64, 1 GPU",
        "value": round(qps32, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt32 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": workload_config(key, W, stats, n) | {
            "layout": "interleaved" if stats["interleaved"] else "per-slot", "tile": args.tile,
            "tuner_trials_ms": tuned["trials"] if tuned else None},
        "roofline": roofline,
        "setup_ms": {"jt_compile_host": round(1e3 * compile_s, 3), "jt_build_and_upload": round(1e3 * build_s, 3)},
        "paths": {
            "fp32_batched": {"queries_per_s": round(qps32, 1),
                             "useful_GBps": round(n * args.steps / dt32 * 3 * T * 4 / 1e9, 1),
                             "kernel_ms_one_profiled_step": {k: round(v[0], 4) for k, v in kinds32.items()},
                             "kernel_share": round(sum(v[0] for v in kinds32.values()) / (1e3 * dt32 / args.steps), 3),
                             "timed_region_events": f"around the dominant kind's launches, in one timed step of every "
                                                    f"{args.event_every}"},
            "fp64_batched": {"queries_per_s": round(qps64b, 1), "slots": n64,
                             "useful_GBps": round(n64 * steps64 / dt64 * 3 * T * 8 / 1e9, 1)},
            "fp64_plain_per_query": {"queries_per_s": round(qps_plain, 1),
                                     "p50_ms": round(1e3 * float(np.median(lat)), 4),
                                     "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 4),
                                     "queries": int(len(lat)), "launch": "hipGraph replay",
                                     "eager_queries_per_s": round(qps_plain_eager, 1),
                                     "eager_p50_ms": round(1e3 * float(np.median(lat_e)), 4)},
            "fp32_plain_per_query": {"queries_per_s": round(qps_plain32, 1),
                                     "p50_ms": round(1e3 * float(np.median(lat32)), 4),
                                     "p99_ms": round(1e3 * float(np.percentile(lat32, 99)), 4),
                                     "queries": int(len(lat32)), "launch": "hipGraph replay"},
            "fp32_batched_with_host_io": {"queries_per_s": round(qps_io, 1)},
            "fp32_vs_fp64_plain": round(qps32 / qps_plain, 2),
        },
    }
    if not args.no_cpu_baseline:
        cb, ojts = cpu_baseline(W, args.cpu_seconds)
        cb["one_core"] = oracle_one_core(ojts, W.sample(20 if len(W.nets) == 1 else 64), lambda j, i: W.cases[j][i])
        out["cpu_baseline"] = cb
        pairs = W.sample(20 if len(W.nets) == 1 else 64)
        forest = len(W.nets) > 1
        mo = W.marg_off

        def batched(post, lp):
            # slot i carries case i of every network
            return lambda j, i: (post[i, mo[j]:mo[j + 1]], None if forest else lp[i])

        def plain_get(j, i):
            idx, post, lp, _ = plain[j]
            k = idx.index(i)
            return post[k], lp[k]

        plain_pairs = [(j, i) for j, i in pairs if j in plain and i in plain[j][0]]
        out["accuracy"] = {
            "fp32_batched": accuracy(W, ojts, batched(post32, lp32), pairs, True),
            "fp64_batched": accuracy(W, ojts, batched(post64, lp64), pairs, False),
            "fp64_plain": accuracy(W, ojts, plain_get, plain_pairs, False),
        }
        if forest:
            out["accuracy"]["fp32_batched"]["max_logpe_err"] = forest_logpe_err(W, ojts, lp32, 0)
            out["accuracy"]["fp64_batched"]["max_logpe_err"] = forest_logpe_err(W, ojts, lp64, 0)
            out["accuracy"]["logpe_note"] = "forest slots: log P(e) of slot 0 against the sum over all networks"
        out["status_nonzero"] = (int(np.count_nonzero(st32)) + int(np.count_nonzero(st64)) +
                                 sum(int(np.count_nonzero(r[3])) for r in plain.values()))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Serving loop: several junction trees resident in device memory, evidence
queries admitted by device-memory footprint and batched per network as they
arrive.

* Residency and admission.  Each network gets one FP32 junction tree whose
  slot count is set by a device-memory budget: the fixed bytes of every tree
  (plan, index maps, prior), the bytes of one FP64 fallback tree, and then as
  many slots per tree as the rest allows (capped at max_batch).  The footprints
  come from host-only builds, which compute exactly what a device build
  allocates, so nothing is allocated past the budget.  A query is admitted when
  a slot of its network's tree is free; until then it waits in that network's
  queue.
* Continuous batching.  Every tree runs on its own stream.  Whenever a tree
  has waiting queries and free slots, and fewer than `depth` batches in
  flight, the waiting queries (up to the free slots) become one batch:
  evidence upload, one calibration (a replayed graph per batch size), and an
  asynchronous copy of the posteriors into pinned host buffers, followed by an
  event.  Completed batches are retired in order when their event has fired;
  their slots become free at once.  Trees of different networks overlap on
  the device.
* Precision.  Table arithmetic in FP32 with rescaled separators; a query whose
  FP32 messages vanish (the underflow flag) is rerun on an FP64 tree of its
  network (built on demand, one at a time, inside the reserve).

Latency is measured from a query's arrival time on the trace clock to the
moment the host sees its batch complete.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import fbn


@dataclass
class Query:
    qid: int
    net: int
    vars: np.ndarray
    states: np.ndarray
    t_arrive: float = 0.0        # seconds on the trace clock


@dataclass
class _Batch:
    qids: list
    slots: list
    post: np.ndarray
    logpe: np.ndarray
    flags: np.ndarray
    event: object
    buf: int


@dataclass
class ServeResult:
    latency: np.ndarray                  # seconds, per query (trace order)
    t_done: np.ndarray
    log_pe: np.ndarray
    status: np.ndarray                   # fbn status per query
    precision: np.ndarray                # FBN_FP32_RESCALED or FBN_FP64 (fallback)
    wall: float                          # first arrival to last completion, seconds
    batches: int
    post: dict = field(default_factory=dict)   # qid -> posteriors, for the kept queries

    @property
    def qps(self) -> float:
        return len(self.latency) / self.wall if self.wall > 0 else 0.0

    def percentile(self, q: float) -> float:
        return float(np.percentile(self.latency, q))


def admission_plan(handles, tiles, budget_bytes: int, max_batch: int, layout: int = 0,
                   shrink_evidence: bool = False, knobs=None) -> dict:
    """Device-memory plan of a server (host only, no device needed): the fixed
    bytes of every tree (plan, maps, prior), one FP64 fallback tree (the
    largest), then as many evidence slots per tree as the rest of the budget
    holds, at most max_batch.  Footprints come from host-only builds, which
    report exactly what a device build allocates.  MemoryError when not even
    one slot per tree fits.  knobs: per tree, the per-slot options
    (slots_per_block, fin_block) its device build will use."""
    fixed, slot, fb = [], [], []
    knobs = knobs or [{}] * len(handles)
    for h, t, kb in zip(handles, tiles, knobs):
        a = fbn.JT(h, host_only=True, precision=fbn.FBN_FP32_RESCALED, max_slots=1, tile_entries=t,
                   layout=layout, shrink_evidence=shrink_evidence, **kb)
        fixed.append(a.stats["device_bytes"] - a.stats["slot_bytes"])
        slot.append(a.stats["slot_bytes"])
        b = fbn.JT(h, host_only=True, precision=fbn.FBN_FP64, max_slots=1, tile_entries=t)
        fb.append(b.stats["device_bytes"])
    reserve = max(fb)
    avail = budget_bytes - sum(fixed) - reserve
    if avail < sum(slot):
        raise MemoryError(f"budget {budget_bytes} B cannot hold every network with one slot "
                          f"(needs {sum(fixed) + reserve + sum(slot)} B)")
    slots = int(min(max_batch, avail // sum(slot)))
    return {"slots": slots, "fixed_bytes": fixed, "slot_bytes": slot, "fallback_reserve": reserve,
            "planned_bytes": sum(fixed) + reserve + slots * sum(slot)}


class Server:
    """Resident FP32 junction trees for `nets` (objects with .flat() and
    .card), one stream each, sized by `budget_bytes`."""

    def __init__(self, nets, budget_bytes: int = 32 << 30, max_batch: int = 32, depth: int = 2,
                 graph: bool = True, tile=0, warm: bool = True, layout: int = 0,
                 tile_candidates=(0, 2048, 4096), shrink_evidence: bool = False, refine: bool = False,
                 batch_cap: int | None = None):
        import torch
        self._torch = torch
        self.nets = list(nets)
        self.card_sum = [int(np.sum(n.card)) for n in self.nets]
        self.layout = layout
        self.depth = max(1, depth)
        handles = [fbn.net_from_spec(n) for n in self.nets]
        # tile per tree: fixed (one for all, or a list with one per tree), or
        # (tile=None) the fastest of tile_candidates for a full batch of
        # max_batch cases, timed on the device, with the tuner's per-slot
        # knobs (slots per workgroup, finaliser block) when `refine`
        self.knobs = [{} for _ in self.nets]
        if isinstance(tile, (list, tuple)):
            if len(tile) != len(self.nets):
                raise ValueError("one tile per network")
            self.tiles = [int(t) for t in tile]
        elif tile is None:
            from . import tune
            empty = (np.zeros(0, np.int32), np.zeros(0, np.int32))
            picks = [tune.tune(n, [empty] * max_batch, fbn.FBN_FP32_RESCALED, max_batch,
                               [(layout or tune.PER_SLOT, t) for t in tile_candidates], reps=3, refine=refine)
                     for n in self.nets]
            self.tiles = [int(r["tile"]) for r in picks]
            self.knobs = [{"slots_per_block": int(r["slots_per_block"]), "fin_block": int(r["fin_block"])}
                          for r in picks]
        else:
            self.tiles = [int(tile)] * len(self.nets)
        self.tile = self.tiles[0]
        plan = admission_plan(handles, self.tiles, budget_bytes, max_batch, layout, shrink_evidence, self.knobs)
        self.slots = plan["slots"]
        # queries per batch at most (default: every free slot)
        self.batch_cap = max(1, min(batch_cap or self.slots, self.slots))
        self.fallback_reserve = plan["fallback_reserve"]
        self.planned_bytes = plan["planned_bytes"]
        self.budget_bytes = budget_bytes
        self.streams = [torch.cuda.Stream() for _ in self.nets]
        self.jts = []
        for h, s, t, kb in zip(handles, self.streams, self.tiles, self.knobs):
            jt = fbn.JT(h, precision=fbn.FBN_FP32_RESCALED, max_slots=self.slots, tile_entries=t,
                        stream=s.cuda_stream, layout=layout, shrink_evidence=shrink_evidence, **kb)
            if graph:
                fbn.set_graph_mode(jt, True)
            self.jts.append(jt)
        self.device_bytes = sum(jt.stats["device_bytes"] for jt in self.jts)
        self._handles = handles
        self._fb = None                      # (network, FP64 jt)
        # pinned result buffers: `depth` per tree
        self._bufs = []
        for k in range(len(self.nets)):
            per = []
            for _ in range(self.depth):
                per.append((torch.empty((self.slots, self.card_sum[k]), dtype=torch.float64, pin_memory=True).numpy(),
                            torch.empty(self.slots, dtype=torch.float64, pin_memory=True).numpy(),
                            torch.empty(self.slots, dtype=torch.int32, pin_memory=True).numpy()))
            self._bufs.append(per)
        if warm:
            self.warm_up()

    def warm_up(self):
        """Capture (graph mode) and run one calibration of every batch size."""
        for k, jt in enumerate(self.jts):
            empty = (np.zeros(0, np.int32), np.zeros(0, np.int32))
            for n in range(1, self.slots + 1):
                sl = list(range(n))
                fbn.set_evidence_batch(jt, sl, [empty] * n)
                fbn.calibrate(jt, sl)
            self.streams[k].synchronize()

    def _fallback(self, net: int):
        if self._fb is None or self._fb[0] != net:
            if self._fb is not None:
                self._fb[1].free()
            self._fb = None
            self._fb = (net, fbn.JT(self._handles[net], precision=fbn.FBN_FP64, max_slots=1,
                                    tile_entries=self.tiles[net]))
        return self._fb[1]

    # ---- device actions of the loop (the scheduling in run() is device-free)
    def _launch(self, k: int, slots, qs, buf: int):
        """Evidence, calibration and an asynchronous read-back of one batch of
        tree k into pinned buffer `buf`; returns the batch's completion event."""
        jt = self.jts[k]
        m = len(slots)
        fbn.set_evidence_batch(jt, slots, [(q.vars, q.states) for q in qs])
        fbn.calibrate(jt, slots)
        post, lp, fl = self._bufs[k][buf]
        fbn.fetch_async(jt, slots, post[:m], lp[:m], fl[:m])
        ev = self._torch.cuda.Event()
        ev.record(self.streams[k])
        return ev

    def _ready(self, k: int, token) -> bool:
        return token.query()

    def _results(self, k: int, buf: int):
        return self._bufs[k][buf]

    def run(self, queries, rate: float | None = None, keep=None) -> ServeResult:
        """Serve `queries` in arrival order.  rate=None: closed loop (every query
        has arrived at t=0); else arrivals at t_arrive / rate seconds.  `keep`:
        query ids whose posteriors are kept in the result.

        Policy: each network keeps its waiting queries in arrival order (FIFO).
        Every pass visits the trees in turn; a tree first retires its finished
        batches (oldest first), then, if it has waiting queries, a free slot and
        a free result buffer (at most `depth` batches in flight), takes the
        oldest waiting queries up to its free slots as one batch.  No tree
        waits on another, so no network starves."""
        n = len(queries)
        order = sorted(range(n), key=lambda i: queries[i].t_arrive)
        arr = np.array([0.0 if rate is None else queries[i].t_arrive / rate for i in range(n)])
        keep = set(keep or ())
        latency = np.full(n, np.nan)
        t_done = np.full(n, np.nan)
        log_pe = np.zeros(n)
        status = np.zeros(n, np.int32)
        prec = np.full(n, fbn.FBN_FP32_RESCALED, np.int32)
        posts = {}
        K = len(self.jts)
        pending = [deque() for _ in range(K)]
        inflight = [deque() for _ in range(K)]
        free = [list(range(self.slots - 1, -1, -1)) for _ in range(K)]
        freebuf = [list(range(self.depth)) for _ in range(K)]
        nxt = 0
        done = 0
        batches = 0
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and arr[order[nxt]] <= now:
                q = queries[order[nxt]]
                pending[q.net].append(order[nxt])
                nxt += 1
            busy = False
            for k in range(K):
                # retire finished batches of tree k, oldest first
                while inflight[k] and self._ready(k, inflight[k][0].event):
                    b = inflight[k].popleft()
                    b.post, b.logpe, b.flags = self._results(k, b.buf)
                    tnow = time.perf_counter() - t0
                    for r, i in enumerate(b.qids):
                        fl = int(b.flags[r])
                        if fl & 2:           # FP32 underflow: rerun in FP64
                            lp, st, post = self._rerun64(queries[i])
                            prec[i] = fbn.FBN_FP64
                            status[i] = st
                            log_pe[i] = lp
                            if i in keep:
                                posts[i] = post
                            tnow = time.perf_counter() - t0
                        else:
                            status[i] = fbn.FBN_E_ZERO_EVIDENCE if fl & 1 else fbn.FBN_OK
                            log_pe[i] = b.logpe[r]
                            if i in keep:
                                posts[i] = b.post[r].copy()
                        t_done[i] = tnow
                        latency[i] = tnow - arr[i]
                    done += len(b.qids)
                    free[k].extend(b.slots)
                    freebuf[k].append(b.buf)
                    busy = True
                # launch a batch from the waiting queries
                if pending[k] and free[k] and freebuf[k]:
                    m = min(len(pending[k]), len(free[k]), self.batch_cap)
                    qids = [pending[k].popleft() for _ in range(m)]
                    slots = [free[k].pop() for _ in range(m)]
                    bi = freebuf[k].pop()
                    ev = self._launch(k, slots, [queries[i] for i in qids], bi)
                    inflight[k].append(_Batch(qids, slots, None, None, None, ev, bi))
                    batches += 1
                    busy = True
            if not busy and nxt < n and not any(inflight):
                # idle until the next arrival
                wait = arr[order[nxt]] - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        wall = float(np.nanmax(t_done) - (0.0 if rate is None else arr.min())) if n else 0.0
        return ServeResult(latency, t_done, log_pe, status, prec, wall, batches, posts)

    def _rerun64(self, q: Query):
        jt = self._fallback(q.net)
        fbn.set_evidence(jt, 0, q.vars, q.states)
        fbn.calibrate(jt, [0])
        post, lp, st = fbn.query_all(jt, [0], self.card_sum[q.net])
        return float(lp[0]), int(st[0]), post[0]

    def close(self):
        for s in self.streams:
            s.synchronize()
        if self._fb is not None:
            self._fb[1].free()
            self._fb = None
        for jt in self.jts:
            jt.free()
        self.jts = []


def serve_plain(nets, queries, rate: float | None = None, graph: bool = True, limit: int | None = None,
                keep=None) -> ServeResult:
    """The per-query FP64 engine on the same trace: one FP64 tree per
    network (one slot), queries taken one at a time in arrival order, each
    waited for before the next (a single FIFO server)."""
    import torch
    nets = list(nets)
    stream = torch.cuda.Stream()
    jts = []
    for net in nets:
        jt = fbn.JT(fbn.net_from_spec(net), precision=fbn.FBN_FP64, max_slots=1, stream=stream.cuda_stream)
        if graph:
            fbn.set_graph_mode(jt, True)
        fbn.set_evidence(jt, 0, np.zeros(0, np.int32), np.zeros(0, np.int32))
        fbn.calibrate(jt, [0], want_results=True)       # warm-up, captures the graph
        jts.append(jt)
    cs = [int(np.sum(n.card)) for n in nets]
    n = len(queries) if limit is None else min(limit, len(queries))
    order = sorted(range(len(queries)), key=lambda i: queries[i].t_arrive)[:n]
    keep = set(keep or ())
    arr = {i: (0.0 if rate is None else queries[i].t_arrive / rate) for i in order}
    latency, t_done, log_pe, status, posts = [], [], [], [], {}
    t0 = time.perf_counter()
    for i in order:
        q = queries[i]
        wait = arr[i] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        jt = jts[q.net]
        fbn.set_evidence(jt, 0, q.vars, q.states)
        fbn.calibrate(jt, [0])
        post, lp, st = fbn.query_all(jt, [0], cs[q.net])
        tnow = time.perf_counter() - t0
        latency.append(tnow - arr[i])
        t_done.append(tnow)
        log_pe.append(float(lp[0]))
        status.append(int(st[0]))
        if i in keep:
            posts[i] = post[0]
    for jt in jts:
        jt.free()
    first = min(arr.values()) if rate is not None and arr else 0.0
    wall = (max(t_done) - first) if t_done else 0.0
    return ServeResult(np.array(latency), np.array(t_done), np.array(log_pe), np.array(status, np.int32),
                       np.full(n, fbn.FBN_FP64, np.int32), wall, n, posts)


def trace_queries(times, which, cases) -> list:
    """Queries of a served-load trace: arrival times (trace clock), the
    network of each arrival and its (vars, states) evidence."""
    return [Query(i, int(which[i]), np.asarray(cases[i][0], np.int32), np.asarray(cases[i][1], np.int32),
                  float(times[i])) for i in range(len(times))]

"""GPU tests of the serving loop on the eight-network served workload:
footprint admission, continuous batching across resident trees, and
served results equal to each query run alone (bitwise: no kernel result
depends on which other slots share a launch), with the FP32 path within its
bar of the oracle and of the plain FP64 engine."""
import numpy as np
import pytest

import fbngen
import oracle
from paper_2212_04241_amd import fbn
from paper_2212_04241_amd.serve import Server, serve_plain, trace_queries
from tests.gpu_util import FP32_ATOL, FP32_LOGPE_ATOL, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c5():
    nets = [fbngen.make_net("C5", j) for j in range(8)]
    times, which, fracs, seeds = fbngen.make_arrivals("C5")
    n = 200
    cases = [fbngen.case_for_arrival(nets[int(which[i])], float(fracs[i]), int(seeds[i])) for i in range(n)]
    return nets, trace_queries(times[:n], which[:n], cases)


def test_host_only_footprint_equals_device_allocation():
    net = fbngen.make_net("C2", 0)
    for prec in (fbn.FBN_FP32_RESCALED, fbn.FBN_FP64):
        a = fbn.JT(fbn.net_from_spec(net), host_only=True, precision=prec, max_slots=5)
        b = fbn.JT(fbn.net_from_spec(net), precision=prec, max_slots=5)
        assert a.stats["device_bytes"] == b.stats["device_bytes"], prec
        assert a.stats["slot_bytes"] == b.stats["slot_bytes"], prec


def test_budget_too_small_is_refused(c5):
    nets, _ = c5
    with pytest.raises(MemoryError):
        Server(nets, budget_bytes=1 << 30, warm=False)


@pytest.mark.timeout(600)
def test_served_mix_equals_alone(c5):
    nets, queries = c5
    say("serve: 8 networks, 200 trace queries")
    srv = Server(nets, budget_bytes=8 << 30, max_batch=6)
    assert srv.slots >= 1 and srv.planned_bytes <= 8 << 30
    assert srv.device_bytes <= srv.planned_bytes - srv.fallback_reserve
    keep = range(len(queries))
    closed = srv.run(queries, None, keep=keep)
    say("closed loop", closed.qps, "q/s,", closed.batches, "batches")
    assert np.all(closed.status == 0) and not np.isnan(closed.latency).any()
    assert closed.batches < len(queries)          # queries were batched
    opened = srv.run(queries, rate=closed.qps * 0.5, keep=keep)
    say("open loop p50/p99 ms", 1e3 * opened.percentile(50), 1e3 * opened.percentile(99))
    srv.close()
    # alone: each query on its own in a fresh one-slot tree of its network
    alone = [fbn.JT(fbn.net_from_spec(n), precision=fbn.FBN_FP32_RESCALED, max_slots=1) for n in nets]
    for i, q in enumerate(queries):
        jt = alone[q.net]
        fbn.set_evidence(jt, 0, q.vars, q.states)
        lp, st = fbn.calibrate(jt, [0], want_results=True)
        post, _, _ = fbn.query_all(jt, [0], int(np.sum(nets[q.net].card)))
        assert st[0] == 0
        for res in (closed, opened):
            assert np.array_equal(res.post[i], post[0]), i
            assert res.log_pe[i] == lp[0], i
    # FP32 against the oracle on the queries of the two smallest networks
    small = [i for i, q in enumerate(queries) if q.net in (6, 7)][:8]
    ojts = {}
    for i in small:
        q = queries[i]
        if q.net not in ojts:
            ojts[q.net] = oracle.compile_net(nets[q.net])
        olp, opost = ojts[q.net].query(q.vars, q.states)
        assert np.max(np.abs(closed.post[i] - opost)) <= FP32_ATOL, i
        assert abs(closed.log_pe[i] - olp) <= FP32_LOGPE_ATOL * max(1.0, abs(olp)), i


@pytest.mark.timeout(600)
def test_plain_fp64_engine_agrees_with_served(c5):
    nets, queries = c5
    qs = queries[:40]
    plain = serve_plain(nets, qs, keep=range(len(qs)))
    assert np.all(plain.status == 0)
    srv = Server(nets, budget_bytes=8 << 30, max_batch=4)
    served = srv.run(qs, None, keep=range(len(qs)))
    srv.close()
    for i in range(len(qs)):
        assert np.max(np.abs(plain.post[i] - served.post[i])) <= FP32_ATOL, i
        assert abs(plain.log_pe[i] - served.log_pe[i]) <= FP32_LOGPE_ATOL * max(1.0, abs(plain.log_pe[i])), i


@pytest.mark.timeout(600)
def test_server_tuned_tiles(c5):
    """Tile per tree picked by timing a full batch of each tree; results are
    bitwise those of a one-slot tree of the same network and tile."""
    nets, queries = c5
    qs = queries[:40]
    srv = Server(nets, budget_bytes=8 << 30, max_batch=4, tile=None, tile_candidates=(0, 2048))
    say("tuned tiles", srv.tiles)
    assert len(srv.tiles) == len(nets) and all(t in (0, 2048) for t in srv.tiles)
    res = srv.run(qs, None, keep=range(len(qs)))
    srv.close()
    assert np.all(res.status == 0)
    for i, q in enumerate(qs):
        jt = fbn.JT(fbn.net_from_spec(nets[q.net]), precision=fbn.FBN_FP32_RESCALED, max_slots=1,
                    tile_entries=srv.tiles[q.net])
        fbn.set_evidence(jt, 0, q.vars, q.states)
        lp, st = fbn.calibrate(jt, [0], want_results=True)
        post, _, _ = fbn.query_all(jt, [0], int(np.sum(nets[q.net].card)))
        jt.free()
        assert st[0] == 0
        assert np.array_equal(res.post[i], post[0]), i
        assert res.log_pe[i] == lp[0], i


def _tiny(text):
    return fbngen.net_from_text(text)


# A -> B with P(B = 1 | A) = 1e-60: observing B = 1 leaves every FP32 table
# entry of the evidence at zero (5e-61 is below float32's range), so the FP32
# path flags underflow and the server reruns the query on an FP64 tree.
_UNDERFLOW_NET = ("fbn 1\nvars 2\nvar 0 2 0\nvar 1 2 1 0\ncpt 0 2\n0.25 0.75\n"
                  "cpt 1 4\n1 1e-60 1 1e-60\nend\n")
# C with P(C = 1) = 0: observing C = 1 has probability zero in any precision.
_ZERO_NET = ("fbn 1\nvars 2\nvar 0 2 0\nvar 1 3 1 0\ncpt 0 2\n1 0\n"
             "cpt 1 6\n0.2 0.3 0.5 0.1 0.1 0.8\nend\n")


@pytest.mark.timeout(600)
def test_served_fp64_fallback():
    from paper_2212_04241_amd.serve import Query
    nets = [_tiny(_UNDERFLOW_NET), _tiny(_ZERO_NET), fbngen.make_net("C1", 0)]
    c1 = fbngen.make_cases("C1", nets[2])[:6]
    qs = [Query(0, 0, np.array([1], np.int32), np.array([1], np.int32)),      # FP32 underflow -> FP64
          Query(1, 2, c1[0][0], c1[0][1]),
          Query(2, 1, np.array([0], np.int32), np.array([1], np.int32)),      # zero evidence
          Query(3, 0, np.array([1], np.int32), np.array([0], np.int32)),      # fine in FP32
          Query(4, 1, np.array([1], np.int32), np.array([2], np.int32))]      # fine in FP32
    qs += [Query(5 + k, 2, c1[k][0], c1[k][1]) for k in range(1, 6)]
    say("served mix with FP64 fallbacks")
    srv = Server(nets, budget_bytes=1 << 30, max_batch=4)
    res = srv.run(qs, None, keep=range(len(qs)))
    tiles = list(srv.tiles)
    srv.close()
    assert res.precision[0] == fbn.FBN_FP64 and res.status[0] == fbn.FBN_OK
    assert res.precision[2] == fbn.FBN_FP64 and res.status[2] == fbn.FBN_E_ZERO_EVIDENCE
    for i in (1, 3, 4) + tuple(range(5, 10)):
        assert res.precision[i] == fbn.FBN_FP32_RESCALED and res.status[i] == fbn.FBN_OK, i
    # the rerun is bitwise the FP64 engine's result for that query alone
    jt = fbn.JT(fbn.net_from_spec(nets[0]), precision=fbn.FBN_FP64, max_slots=1, tile_entries=tiles[0])
    fbn.set_evidence(jt, 0, qs[0].vars, qs[0].states)
    lp, st = fbn.calibrate(jt, [0], want_results=True)
    post, _, _ = fbn.query_all(jt, [0], int(np.sum(nets[0].card)))
    assert st[0] == 0
    assert np.array_equal(res.post[0], post[0]) and res.log_pe[0] == lp[0]
    # and the oracle's: P(A | B = 1) = P(A), P(e) = 1e-60
    ojt = oracle.compile_net(nets[0])
    olp, opost = ojt.query(qs[0].vars, qs[0].states)
    assert np.all(np.abs(res.post[0] - opost) <= 1e-12 * np.abs(opost))
    assert abs(res.log_pe[0] - olp) <= 1e-12 * abs(olp)
    assert abs(olp - np.log(1e-60)) <= 1e-12 * abs(olp)


@pytest.mark.timeout(600)
def test_second_batch_of_a_tree_is_enqueued_while_the_first_runs():
    """After calibrate + fetch_async of one batch, entering the next batch's
    evidence returns without waiting for the first calibration."""
    import torch
    net = fbngen.make_net("C3", 0)
    cases = fbngen.make_cases("C3", net)[:8]
    s = torch.cuda.Stream()
    jt = fbn.JT(fbn.net_from_spec(net), precision=fbn.FBN_FP32_RESCALED, max_slots=8, stream=s.cuda_stream)
    cs = int(np.sum(net.card))
    bufs = [(torch.empty((4, cs), dtype=torch.float64, pin_memory=True).numpy(),
             torch.empty(4, dtype=torch.float64, pin_memory=True).numpy(),
             torch.empty(4, dtype=torch.int32, pin_memory=True).numpy()) for _ in range(2)]
    a, b = [0, 1, 2, 3], [4, 5, 6, 7]
    for _ in range(2):     # warm up, then the timed pattern
        fbn.set_evidence_batch(jt, a, cases[:4])
        fbn.calibrate(jt, a)
        fbn.fetch_async(jt, a, *bufs[0])
        e1 = torch.cuda.Event()
        e1.record(s)
        fbn.set_evidence_batch(jt, b, cases[4:])
        queued = not e1.query()
        fbn.calibrate(jt, b)
        fbn.fetch_async(jt, b, *bufs[1])
        s.synchronize()
    say("second batch entered while the first ran:", queued)
    assert queued
    # results of both batches are those of the same cases run alone
    for buf, ids in ((bufs[0], range(4)), (bufs[1], range(4, 8))):
        assert not buf[2].any()
        one = fbn.JT(fbn.net_from_spec(net), precision=fbn.FBN_FP32_RESCALED, max_slots=1)
        for r, k in enumerate(ids):
            fbn.set_evidence(one, 0, *cases[k])
            fbn.calibrate(one, [0])
            post, lp, _ = fbn.query_all(one, [0], cs)
            assert np.array_equal(buf[0][r], post[0]) and buf[1][r] == lp[0], k
        one.free()
    jt.free()


@pytest.mark.timeout(900)
def test_served_fp32_matches_oracle_on_200_trace_queries(c5):
    """The served FP32 path in the configuration the benchmark times (64
    slots per tree in a 64 GiB budget, tile 2048 on every tree) against the
    oracle on the first 200 queries of the arrival trace, every posterior
    entry."""
    from concurrent.futures import ThreadPoolExecutor
    nets, queries = c5
    srv = Server(nets, budget_bytes=64 << 30, max_batch=64, tile=[2048] * len(nets))
    assert srv.slots == 64
    res = srv.run(queries, None, keep=range(len(queries)))
    srv.close()
    assert np.all(res.status == 0)
    ojts = {}
    with ThreadPoolExecutor(8) as ex:
        for k, o in zip(range(8), ex.map(lambda k: oracle.compile_net(nets[k]), range(8))):
            ojts[k] = o
        ref = list(ex.map(lambda q: ojts[q.net].query(q.vars, q.states), queries))
    worst = 0.0
    for i, (olp, opost) in enumerate(ref):
        e = float(np.max(np.abs(res.post[i] - opost)))
        worst = max(worst, e)
        assert e <= FP32_ATOL, (i, e)
        assert abs(res.log_pe[i] - olp) <= FP32_LOGPE_ATOL * max(1.0, abs(olp)), i
    say("served fp32 worst abs error over", len(ref), "queries:", worst)

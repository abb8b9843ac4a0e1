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

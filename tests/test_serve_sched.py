"""The serving loop's host policy on the CPU, with a fake executor in place of
the device: memory-budget admission (from host-only footprints), per-network
FIFO batching, no starvation across networks, slot and buffer accounting, and
the FP64 rerun of an underflowed query.  The loop's scheduling is the same
code that drives the GPU; only the three device actions are replaced."""
import numpy as np
import pytest

import fbngen
from paper_2212_04241_amd import fbn
from paper_2212_04241_amd.serve import Query, Server, admission_plan


class FakeServer(Server):
    """Server with a fake device: a batch completes after `polls` readiness
    checks; its posteriors are (qid, slot) stamps; flags come from `flags`."""

    def __init__(self, n_nets, slots, depth=2, polls=2, flags=None, card_sum=4, batch_cap=None):
        self.nets = [None] * n_nets
        self.card_sum = [card_sum] * n_nets
        self.jts = [None] * n_nets
        self.slots = slots
        self.batch_cap = batch_cap or slots
        self.depth = depth
        self.polls = polls
        self.flags = flags or {}
        self._bufs = [[(np.zeros((slots, card_sum)), np.zeros(slots), np.zeros(slots, np.int32))
                       for _ in range(depth)] for _ in range(n_nets)]
        self.launches = []          # (tree, slots, qids) in launch order
        self.inflight_slots = [set() for _ in range(n_nets)]
        self.max_inflight_batches = [0] * n_nets
        self._live = [0] * n_nets
        self.reruns = []

    def _launch(self, k, slots, qs, buf):
        assert not (set(slots) & self.inflight_slots[k]), "slot reused while in flight"
        self.inflight_slots[k] |= set(slots)
        self._live[k] += 1
        self.max_inflight_batches[k] = max(self.max_inflight_batches[k], self._live[k])
        post, lp, fl = self._bufs[k][buf]
        for r, (s, q) in enumerate(zip(slots, qs)):
            post[r] = [q.qid, s, k, 0]
            lp[r] = -float(q.qid)
            fl[r] = self.flags.get(q.qid, 0)
        self.launches.append((k, list(slots), [q.qid for q in qs]))
        return {"left": self.polls, "slots": list(slots)}

    def _ready(self, k, token):
        token["left"] -= 1
        if token["left"] <= 0:
            self.inflight_slots[k] -= set(token["slots"])
            self._live[k] -= 1
            return True
        return False

    def _rerun64(self, q):
        self.reruns.append(q.qid)
        return -1000.0 - q.qid, fbn.FBN_OK, np.full(self.card_sum[q.net], 0.25)


def _queries(nets_of, t=None):
    return [Query(i, k, np.zeros(0, np.int32), np.zeros(0, np.int32), 0.0 if t is None else t[i])
            for i, k in enumerate(nets_of)]


def test_every_query_served_once_in_fifo_order_per_network():
    rng = np.random.default_rng(0)
    nets_of = rng.integers(0, 3, size=200)
    srv = FakeServer(3, slots=4)
    res = srv.run(_queries(nets_of), None, keep=range(200))
    served = [q for _, _, qids in srv.launches for q in qids]
    assert sorted(served) == list(range(200))
    for k in range(3):
        mine = [q for kk, _, qids in srv.launches if kk == k for q in qids]
        assert mine == [i for i in range(200) if nets_of[i] == k]      # arrival order
    assert np.all(res.status == 0) and not np.isnan(res.latency).any()
    for i in range(200):                                                 # results routed back
        assert res.post[i][0] == i and res.log_pe[i] == -i


def test_slots_and_buffers_never_oversubscribed():
    srv = FakeServer(2, slots=3, depth=2, polls=3)
    srv.run(_queries([0] * 50 + [1] * 50), None)
    for k, slots, qids in srv.launches:
        assert 1 <= len(slots) <= 3 and len(set(slots)) == len(slots)
    assert max(srv.max_inflight_batches) <= 2


def test_batch_cap_splits_a_backlog_into_batches_in_flight_together():
    srv = FakeServer(1, slots=8, depth=2, polls=4, batch_cap=4)
    srv.run(_queries([0] * 40), None)
    assert all(len(slots) <= 4 for _, slots, _ in srv.launches)
    assert srv.max_inflight_batches[0] == 2          # two half-size batches overlap
    served = [q for _, _, qids in srv.launches for q in qids]
    assert served == list(range(40))
    # without the cap one batch takes every free slot, so a second cannot start
    srv = FakeServer(1, slots=8, depth=2, polls=4)
    srv.run(_queries([0] * 40), None)
    assert srv.max_inflight_batches[0] == 1 and len(srv.launches[0][1]) == 8


def test_no_network_starves_behind_a_backlog():
    # network 0 has a flood, network 1 a single query: it is launched in the
    # first pass, before most of the flood
    nets_of = [0] * 300 + [1]
    srv = FakeServer(2, slots=2, polls=5)
    srv.run(_queries(nets_of), None)
    first_one = next(i for i, (k, _, _) in enumerate(srv.launches) if k == 1)
    assert first_one <= 2
    # open loop: a late query of network 1 waits at most one batch of network 0
    t = np.concatenate([np.zeros(300), [1e-4]])
    srv = FakeServer(2, slots=2, polls=5)
    srv.run(_queries(nets_of, t), rate=1.0)
    k1 = next(i for i, (k, _, _) in enumerate(srv.launches) if k == 1)
    assert all(k == 0 for k, _, _ in srv.launches[:k1])


def test_underflowed_query_is_rerun_in_fp64_and_zero_evidence_reported():
    srv = FakeServer(2, slots=4, flags={3: 2, 7: 1, 8: 2})
    res = srv.run(_queries([0, 1] * 6), None, keep=range(12))
    assert sorted(srv.reruns) == [3, 8]
    assert res.precision[3] == fbn.FBN_FP64 and res.log_pe[3] == -1003.0
    assert np.all(res.post[3] == 0.25)
    assert res.status[7] == fbn.FBN_E_ZERO_EVIDENCE and res.precision[7] == fbn.FBN_FP32_RESCALED
    assert all(res.precision[i] == fbn.FBN_FP32_RESCALED for i in range(12) if i not in (3, 8))


def test_admission_plan_stays_inside_the_budget():
    nets = [fbngen.make_net("C1", 0), fbngen.make_net("C2", 0)]
    handles = [fbn.net_from_spec(n) for n in nets]
    plans = {}
    for gib in (0.05, 0.2, 1.0):
        budget = int(gib * (1 << 30))
        p = admission_plan(handles, [0, 0], budget, max_batch=1000)
        assert p["planned_bytes"] <= budget
        # one more slot per tree would not fit (or max_batch caps it)
        assert p["slots"] == 1000 or p["planned_bytes"] + sum(p["slot_bytes"]) > budget
        plans[gib] = p["slots"]
    assert plans[0.05] <= plans[0.2] <= plans[1.0]
    with pytest.raises(MemoryError):
        admission_plan(handles, [0, 0], 1 << 20, max_batch=8)

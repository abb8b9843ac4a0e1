"""GPU parity of the multi-network batch: many independent networks in one
forest junction tree, one slot carrying a case of every network.  Each
network's slice of the posteriors is checked against the oracle run on that
network alone; the slot's log P(e) against the sum of the oracle's per
network (the networks are independent, so P(e) factorises)."""
import numpy as np
import pytest

import fbngen
import oracle
from paper_2212_04241_amd import fbn
from tests.gpu_util import FP32_ATOL, FP32_LOGPE_ATOL, FP64_RTOL, say

pytestmark = pytest.mark.gpu


def _forest(n_nets):
    nets = [fbngen.make_net("C4", j) for j in range(n_nets)]
    cases = [fbngen.make_cases("C4", n, j) for j, n in enumerate(nets)]
    return nets, cases, fbngen.forest_offsets(nets)


def _marg_offsets(nets):
    return np.concatenate([[0], np.cumsum([int(np.sum(n.card)) for n in nets])])


def _run(jt, nets, cases, off, slots, case_ids, graph=False):
    fbn.set_evidence_batch(jt, slots, [fbngen.forest_case(off, cases, s) for s in case_ids])
    fbn.calibrate(jt, slots)
    return fbn.query_all(jt, slots, int(sum(int(np.sum(n.card)) for n in nets)))


def _check(nets, cases, post, lp, st, case_ids, check_nets, lp_nets, fp32):
    mo = _marg_offsets(nets)
    ojts = {}

    def ojt_of(k):
        if k not in ojts:
            ojts[k] = oracle.compile_net(nets[k])
        return ojts[k]

    assert np.all(st == 0), st
    worst = 0.0
    for k in check_nets:
        ojt = ojt_of(k)
        for b, s in enumerate(case_ids):
            _, opost = ojt.query(*cases[k][s])
            got = post[b, mo[k]:mo[k + 1]]
            err = np.abs(got - opost)
            if fp32:
                worst = max(worst, float(err.max()))
                assert err.max() <= FP32_ATOL, (k, s, float(err.max()))
            else:
                assert np.all(err <= FP64_RTOL * np.abs(opost) + 1e-300), (k, s)
    for b in lp_nets:
        s = case_ids[b]
        olp = 0.0
        for k in range(len(nets)):
            l, _ = ojt_of(k).query(*cases[k][s])
            olp += l
        tol = (FP32_LOGPE_ATOL if fp32 else FP64_RTOL) * max(1.0, abs(olp))
        assert abs(lp[b] - olp) <= tol, (b, lp[b], olp)
    return worst


def test_forest_fp64_16_networks():
    nets, cases, off = _forest(16)
    say("forest fp64, 16 networks x 8 cases")
    jt = fbn.JT([fbn.net_from_spec(n) for n in nets], precision=fbn.FBN_FP64, max_slots=8)
    assert jt.stats["n_trees"] == 16
    ids = list(range(8))
    post, lp, st = _run(jt, nets, cases, off, ids, ids)
    _check(nets, cases, post, lp, st, ids, range(16), [0, 7], fp32=False)


def test_forest_fp64_mixed_shapes():
    # very uneven trees side by side: a one-clique network, a disconnected
    # one, a deep C2-shaped one and small random ones
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden", "micro")
    nets = []
    for name in ("one_node.fbn", "disconnected.fbn"):
        with open(os.path.join(gold, name)) as f:
            nets.append(fbngen.net_from_text(f.read()))
    nets.append(fbngen.make_net("C2", 0))
    nets += [fbngen.random_small_net(s, 14, max_card=4, window=6) for s in (1, 2)]
    rng = np.random.default_rng(5)
    cases = []
    for n in nets:
        cs = []
        for _ in range(4):
            m = int(rng.integers(0, max(1, n.n // 5) + 1))
            vs = np.sort(rng.choice(n.n, size=m, replace=False)).astype(np.int32)
            cs.append((vs, np.array([int(rng.integers(0, int(n.card[v]))) for v in vs], np.int32)))
        cases.append(cs)
    off = fbngen.forest_offsets(nets)
    say("forest fp64, mixed shapes")
    for tile in (0, 100):
        jt = fbn.JT([fbn.net_from_spec(n) for n in nets], precision=fbn.FBN_FP64, max_slots=4, tile_entries=tile)
        ids = [0, 1, 2, 3]
        post, lp, st = _run(jt, nets, cases, off, [3, 1, 0, 2], ids)
        _check(nets, cases, post, lp, st, ids, range(len(nets)), [0, 1, 2, 3], fp32=False)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("layout,tile", [(fbn.FBN_LAYOUT_PER_SLOT, 0), (fbn.FBN_LAYOUT_INTERLEAVED, 128)])
def test_forest_c4_full_batch_fp32_graph(layout, tile):
    # the full batch: 256 networks x 64 cases in one calibration, FP32,
    # replayed from a captured graph; posteriors of a sample of 16 networks
    # (every case), log P(e) of three slots over all 256 networks.  The
    # interleaved layout at tile 128 is the configuration the bench times.
    import torch
    nets, cases, off = _forest(256)
    say("forest fp32, 256 networks x 64 cases, graph, layout", layout, "tile", tile)
    s = torch.cuda.Stream()
    jt = fbn.JT([fbn.net_from_spec(n) for n in nets], precision=fbn.FBN_FP32_RESCALED, max_slots=64,
                stream=s.cuda_stream, layout=layout, tile_entries=tile)
    fbn.set_graph_mode(jt, True)
    ids = list(range(64))
    for rep in range(2):
        post, lp, st = _run(jt, nets, cases, off, ids, ids)
        if rep == 0:
            first = (post.copy(), lp.copy())
    assert np.array_equal(first[0], post) and np.array_equal(first[1], lp)
    sample = list(range(8)) + [31, 63, 100, 127, 160, 200, 254, 255]
    worst = _check(nets, cases, post, lp, st, ids, sample, [0, 31, 63], fp32=True)
    say("worst fp32 abs error", worst)
    del jt
    torch.cuda.synchronize()


@pytest.mark.timeout(600)
def test_forest_c4g_unrepaired_draws_fp32():
    # networks drawn by rejection under the 4e6-entry guard, every drawn arc
    # kept: the first 16 as one forest, FP32 interleaved at tile 256 (the
    # bench's configuration for this batch); posteriors of four networks and
    # log P(e) of two slots against the oracle
    nets = [fbngen.make_net("C4G", j) for j in range(16)]
    cases = [fbngen.make_cases("C4G", n, j, n_cases=8) for j, n in enumerate(nets)]
    off = fbngen.forest_offsets(nets)
    say("forest C4G fp32, 16 networks x 8 cases, T", sum(oracle.compile_net(n, structure_only=True).T for n in nets))
    jt = fbn.JT([fbn.net_from_spec(n) for n in nets], precision=fbn.FBN_FP32_RESCALED, max_slots=8,
                layout=fbn.FBN_LAYOUT_INTERLEAVED, tile_entries=256)
    ids = list(range(8))
    post, lp, st = _run(jt, nets, cases, off, ids, ids)
    worst = _check(nets, cases, post, lp, st, ids, [0, 3, 9, 15], [0, 5], fp32=True)
    say("worst fp32 abs error", worst)
    jt.free()

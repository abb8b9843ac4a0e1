"""GPU parity of the slot-interleaved layout (entry x of slot s at
x * max_slots + s, one lane per slot) against the FP64 oracle, with the same
bars as the per-slot layout, plus its own invariants: a slot's result is
bitwise the same whichever other slots share the launch, and a replayed
graph equals eager launches."""
import os

import numpy as np
import pytest

import fbngen
from paper_2212_04241_amd import fbn
from tests.gpu_util import check_fp32, check_fp64, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu

IL = fbn.FBN_LAYOUT_INTERLEAVED
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "micro")


def _cases(net, k, n_obs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        m = min(n_obs, net.n)
        vs = np.sort(rng.choice(net.n, size=m, replace=False)).astype(np.int32)
        ss = np.array([int(rng.integers(0, int(net.card[v]))) for v in vs], dtype=np.int32)
        out.append((vs, ss))
    return out


def test_layout_is_reported():
    net = fbngen.make_net("C1", 0)
    assert fbn.JT(fbn.net_from_spec(net), max_slots=40).stats["interleaved"] == 0
    assert fbn.JT(fbn.net_from_spec(net), max_slots=8).stats["interleaved"] == 0
    assert fbn.JT(fbn.net_from_spec(net), max_slots=8, layout=IL).stats["interleaved"] == 1
    assert fbn.JT(fbn.net_from_spec(net), max_slots=40, layout=fbn.FBN_LAYOUT_PER_SLOT).stats["interleaved"] == 0


@pytest.mark.parametrize("seed", range(6))
def test_random_nets(seed):
    say("interleaved random", seed)
    net = fbngen.random_small_net(3000 + seed, 25 + 5 * seed, max_card=4, p_max=3, window=6, alpha=0.5)
    cases = _cases(net, 9, 1 + seed, seed) + [(np.zeros(0, np.int32), np.zeros(0, np.int32))]
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases, layout=IL)
    check_fp64(post, lp, st, ref, f"il fp64 {seed}")
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED, layout=IL)
    check_fp32(post, lp, st, ref, f"il fp32 {seed}")


def test_c1_all_cases():
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)
    say("interleaved C1", len(cases))
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases, layout=IL)
    check_fp64(post, lp, st, ref, "il C1")
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED, layout=IL)
    check_fp32(post, lp, st, ref, "il C1 fp32")


@pytest.mark.parametrize("tile", [37, 256, 1000])
def test_c2_ragged_tiles(tile):
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:20]
    say("interleaved C2 tile", tile)
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases, tile=tile, layout=IL)
    check_fp64(post, lp, st, ref, f"il C2 tile {tile}")
    post, lp, st, _ = gpu_run(net, cases, tile=tile, precision=fbn.FBN_FP32_RESCALED, layout=IL)
    say("worst fp32", check_fp32(post, lp, st, ref, f"il C2 fp32 tile {tile}"))


@pytest.mark.timeout(600)
def test_c3_huge_clique():
    net = fbngen.make_net("C3", 0)
    cases = fbngen.make_cases("C3", net)[:3]
    say("interleaved C3")
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases[:2], layout=IL)
    check_fp64(post, lp, st, ref[:2], "il C3 fp64")
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED, layout=IL)
    say("worst fp32", check_fp32(post, lp, st, ref, "il C3 fp32"))


@pytest.mark.timeout(600)
def test_c3_bench_subset_fp32():
    # the bench's C3 configuration (interleaved, tile 256, FP32) on the first
    # 20 cases, every posterior entry against the oracle
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    net = fbngen.make_net("C3", 0)
    cases = fbngen.make_cases("C3", net)[:20]
    ojt = oracle.compile_net(net)
    say("interleaved C3 fp32, 20 cases, tile 256")
    with ThreadPoolExecutor(8) as ex:
        ref = list(ex.map(lambda c: ojt.query(*c), cases))
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED, layout=IL, tile=256)
    say("worst fp32", check_fp32(post, lp, st, ref, "il C3 fp32 bench subset"))


@pytest.mark.timeout(600)
def test_c5_network():
    net = fbngen.make_net("C5", 7)
    rng = np.random.default_rng(11)
    cases = [fbngen.case_for_arrival(net, f, int(rng.integers(0, 2**62))) for f in (0.02, 0.1, 0.2)]
    say("interleaved C5 net 7")
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases, layout=IL)
    check_fp64(post, lp, st, ref, "il C5 fp64")
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED, layout=IL)
    check_fp32(post, lp, st, ref, "il C5 fp32")


def test_degenerate_and_zero_evidence():
    for name in ["one_node.fbn", "disconnected.fbn"]:
        with open(os.path.join(GOLDEN, name)) as f:
            net = fbngen.net_from_text(f.read())
        say("interleaved degenerate", name)
        cases = [(np.zeros(0, np.int32), np.zeros(0, np.int32))] + \
                [(np.array([v], np.int32), np.array([int(net.card[v]) - 1], np.int32)) for v in range(net.n)]
        ref, _ = oracle_run(net, cases)
        post, lp, st, _ = gpu_run(net, cases, layout=IL)
        check_fp64(post, lp, st, ref, name)
    text = ("fbn 1\nvars 3\nvar 0 2 0\nvar 1 2 1 0\nvar 2 2 1 1\ncpt 0 2\n1 0\ncpt 1 4\n1 0 0.5 0.5\n"
            "cpt 2 4\n0.5 0.5 0.25 0.75\nend\n")
    net = fbngen.net_from_text(text)
    cases = [(np.array([1], np.int32), np.array([1], np.int32)), (np.array([2], np.int32), np.array([1], np.int32))]
    ref1, _ = oracle_run(net, [cases[1]])
    post, lp, st, _ = gpu_run(net, cases, layout=IL)
    assert st[0] == fbn.FBN_E_ZERO_EVIDENCE and lp[0] == -np.inf
    check_fp64(post[1:], lp[1:], st[1:], ref1, "il neighbour slot")
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED, layout=IL)
    assert st[0] == fbn.FBN_E_UNDERFLOW and st[1] == 0


@pytest.mark.parametrize("prec", [fbn.FBN_FP64, fbn.FBN_FP32_RESCALED])
def test_slot_independence_bitwise(prec):
    # the same case gives bitwise the same result in a full batch, alone,
    # and at another slot among other cases
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:70]
    say("interleaved slot independence", prec)
    marg = int(np.sum(net.card))
    jt = fbn.JT(fbn.net_from_spec(net), precision=prec, max_slots=72, layout=IL)
    post_b, lp_b, st_b, _ = gpu_run(net, cases, jt=jt)
    assert np.all(st_b == 0)
    for k in (0, 33, 69):
        fbn.set_evidence(jt, 71, *cases[k])
        lp1, _ = fbn.calibrate(jt, [71], want_results=True)
        p1, _, _ = fbn.query_all(jt, [71], marg)
        assert np.array_equal(p1[0], post_b[k]) and lp1[0] == lp_b[k], k
    # scattered slots, another order
    order = [5, 64, 2, 70, 31]
    fbn.set_evidence_batch(jt, order, [cases[k] for k in (10, 11, 12, 13, 14)])
    fbn.calibrate(jt, order)
    p2, l2, _ = fbn.query_all(jt, order, marg)
    for j, k in enumerate((10, 11, 12, 13, 14)):
        assert np.array_equal(p2[j], post_b[k]) and l2[j] == lp_b[k], k


def test_graph_replay_equals_eager():
    import torch
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:96]
    say("interleaved graph replay")
    marg = int(np.sum(net.card))
    eager = fbn.JT(fbn.net_from_spec(net), precision=fbn.FBN_FP32_RESCALED, max_slots=48, layout=IL)
    s = torch.cuda.Stream()
    graph = fbn.JT(fbn.net_from_spec(net), precision=fbn.FBN_FP32_RESCALED, max_slots=48, layout=IL,
                   stream=s.cuda_stream)
    fbn.set_graph_mode(graph, True)
    slots = list(range(48))
    for rep in range(2):
        batch = cases[48 * rep: 48 * rep + 48]
        fbn.set_evidence_batch(eager, slots, batch)
        fbn.set_evidence_batch(graph, slots, batch)
        fbn.calibrate(eager, slots)
        pe, le, se = fbn.query_all(eager, slots, marg)
        fbn.calibrate(graph, slots)
        pg, lg, sg = fbn.query_all(graph, slots, marg)
        torch.cuda.synchronize()
        assert np.array_equal(pe, pg) and np.array_equal(le, lg) and np.array_equal(se, sg), rep
    ref, _ = oracle_run(net, cases[48:60])
    check_fp32(pg[:12], lg[:12], sg[:12], ref, "il graph")
    del graph
    torch.cuda.synchronize()


def test_tuner_choice_keeps_parity(tmp_path):
    from paper_2212_04241_amd import tune
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:24]
    say("tuner on C2")
    r = tune.tune(net, cases, cache=str(tmp_path / "t.json"),
                  candidates=[(tune.PER_SLOT, 0), (tune.PER_SLOT, 2048), (tune.INTERLEAVED, 128)])
    # the choice is within the tuner's 2% tolerance of the fastest trial
    assert len(r["trials"]) == 3 and r["ms"] <= min(t[2] for t in r["trials"]) * 1.02 + 1e-12
    ref, _ = oracle_run(net, cases[:8])
    post, lp, st, _ = gpu_run(net, cases[:8], precision=fbn.FBN_FP32_RESCALED, tile=r["tile"], layout=r["layout"])
    check_fp32(post, lp, st, ref, "tuned")

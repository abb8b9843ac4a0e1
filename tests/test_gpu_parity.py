"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Bars: index maps bit-exact; FP64 posteriors and P(e)
within 1e-12 relative per entry; FP32 posteriors within 1e-5 absolute."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import fbngen
import oracle
from paper_2212_04241_amd import fbn
from tests.gpu_util import (FP32_ATOL, check_fp32, check_fp64, gpu_run, oracle_run, say)

pytestmark = pytest.mark.gpu

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


# ------------------------------------------------------------------ maps

@pytest.mark.parametrize("key", ["C1", "C2"])
def test_device_index_maps_bit_exact(key):
    say("device maps", key)
    net = fbngen.make_net(key, 0)
    ojt = oracle.compile_net(net)
    jt = fbn.JT(fbn.net_from_spec(net))
    for e in range(ojt.n_edges):
        assert np.array_equal(fbn.jt_device_index_map(jt, e, net.card), ojt.index_map(e)), e


# ------------------------------------------------------------------ FP64

def test_micro_nets_exact_fractions_fp64():
    with open(os.path.join(GOLDEN, "expected.json")) as f:
        spec = json.load(f)
    for case in spec["cases"]:
        say("micro", case["net"], case["evidence"])
        with open(os.path.join(GOLDEN, case["net"])) as f:
            net = fbngen.net_from_text(f.read())
        ev = case["evidence"]
        cases = [(np.array([v for v, _ in ev], np.int32), np.array([s for _, s in ev], np.int32))]
        post, lp, st, _ = gpu_run(net, cases)
        assert st[0] == 0
        want = np.array([float(Fraction(x)) for row in case["post"] for x in row])
        assert np.max(np.abs(post[0] - want)) <= 1e-15
        pe = float(Fraction(case["pe"]))
        assert abs(np.exp(lp[0]) - pe) <= 1e-14 * pe


@pytest.mark.parametrize("seed", range(8))
def test_random_nets_fp64(seed):
    say("random fp64", seed)
    net = fbngen.random_small_net(1000 + seed, 30 + 5 * seed, max_card=4, p_max=3, window=6, alpha=0.5)
    cases = _cases(net, 7, 1 + seed, seed) + [(np.zeros(0, np.int32), np.zeros(0, np.int32))]
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases)
    check_fp64(post, lp, st, ref, f"seed {seed}")


def test_c1_all_cases_fp64_batched_and_one_by_one():
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)
    say("C1 fp64 batched", len(cases))
    ref, ojt = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases)
    check_fp64(post, lp, st, ref, "C1 batch")
    say("C1 fp64 one slot, sequential")
    jt = fbn.JT(fbn.net_from_spec(net), max_slots=1)
    for k, c in enumerate(cases[:25]):
        p1, l1, s1, _ = gpu_run(net, [c], jt=jt)
        check_fp64(p1, l1, s1, [ref[k]], f"C1 single {k}")


@pytest.mark.parametrize("tile", [64, 100, 333, 4096])
def test_c2_fp64_ragged_tiles(tile):
    # small tiles force segments split across workgroups (partial sums) and
    # tiles that are not a multiple of the segment length
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:6]
    say("C2 fp64 tile", tile)
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases, tile=tile)
    check_fp64(post, lp, st, ref, f"C2 tile {tile}")


def test_c2_first_20_cases_fp64():
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:20]
    say("C2 fp64 20 cases")
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases)
    check_fp64(post, lp, st, ref, "C2")


# ------------------------------------------------------------------ FP32

def test_c1_fp32():
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)
    say("C1 fp32", len(cases))
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED)
    say("C1 fp32 worst abs error", check_fp32(post, lp, st, ref, "C1 fp32"))


@pytest.mark.parametrize("tile", [100, 0])
def test_c2_fp32(tile):
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:20]
    say("C2 fp32 tile", tile)
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED, tile=tile)
    say("C2 fp32 worst abs error", check_fp32(post, lp, st, ref, "C2 fp32"))


@pytest.mark.parametrize("seed", range(4))
def test_random_nets_fp32(seed):
    net = fbngen.random_small_net(2000 + seed, 40, max_card=5, p_max=3, window=5, alpha=0.3)
    cases = _cases(net, 6, 8, seed)
    say("random fp32", seed)
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED)
    check_fp32(post, lp, st, ref, f"fp32 seed {seed}")


@pytest.fixture(scope="module")
def c3():
    net = fbngen.make_net("C3", 0)
    cases = fbngen.make_cases("C3", net)[:4]
    ref, ojt = oracle_run(net, cases)
    return net, cases, ref


@pytest.mark.timeout(600)
def test_c3_huge_clique_fp64(c3):
    # ~1.3e7-entry clique: segments and gathers split across workgroups
    net, cases, ref = c3
    say("C3 fp64", len(cases[:2]))
    post, lp, st, _ = gpu_run(net, cases[:2])
    check_fp64(post, lp, st, ref[:2], "C3 fp64")


@pytest.mark.timeout(600)
def test_c3_huge_clique_fp32(c3):
    net, cases, ref = c3
    say("C3 fp32", len(cases))
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED)
    say("C3 fp32 worst abs error", check_fp32(post, lp, st, ref, "C3 fp32"))


@pytest.mark.timeout(600)
def test_c5_network_fp64_and_fp32():
    net = fbngen.make_net("C5", 7)
    rng = np.random.default_rng(7)
    cases = []
    for k in range(3):
        seed = int(rng.integers(0, 2**62))
        cases.append(fbngen.case_for_arrival(net, [0.02, 0.1, 0.2][k], seed))
    say("C5 net 7", net.n)
    ref, _ = oracle_run(net, cases)
    post, lp, st, _ = gpu_run(net, cases)
    check_fp64(post, lp, st, ref, "C5 fp64")
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED)
    say("C5 fp32 worst abs error", check_fp32(post, lp, st, ref, "C5 fp32"))


# ------------------------------------------------------------------ edge cases

def test_degenerate_networks():
    for name in ["one_node.fbn", "disconnected.fbn"]:
        with open(os.path.join(GOLDEN, name)) as f:
            net = fbngen.net_from_text(f.read())
        say("degenerate", name)
        cases = [(np.zeros(0, np.int32), np.zeros(0, np.int32))] + \
                [(np.array([v], np.int32), np.array([int(net.card[v]) - 1], np.int32)) for v in range(net.n)]
        ref, _ = oracle_run(net, cases)
        for prec in (fbn.FBN_FP64, fbn.FBN_FP32_RESCALED):
            post, lp, st, _ = gpu_run(net, cases, precision=prec)
            (check_fp64 if prec == fbn.FBN_FP64 else check_fp32)(post, lp, st, ref, name)


def test_all_variables_observed():
    net = fbngen.make_net("C1", 0)
    rng = np.random.default_rng(0)
    vs = np.arange(net.n, dtype=np.int32)
    ss = np.array([int(rng.integers(0, int(net.card[v]))) for v in vs], np.int32)
    say("all observed")
    ref, _ = oracle_run(net, [(vs, ss)])
    post, lp, st, _ = gpu_run(net, [(vs, ss)])
    check_fp64(post, lp, st, ref, "all observed")


def test_zero_probability_evidence_flags_slot_only():
    text = ("fbn 1\nvars 3\nvar 0 2 0\nvar 1 2 1 0\nvar 2 2 1 1\ncpt 0 2\n1 0\ncpt 1 4\n1 0 0.5 0.5\n"
            "cpt 2 4\n0.5 0.5 0.25 0.75\nend\n")
    net = fbngen.net_from_text(text)
    cases = [(np.array([1], np.int32), np.array([1], np.int32)),      # P(e) = 0
             (np.array([2], np.int32), np.array([1], np.int32))]      # fine
    say("zero evidence")
    ref1, _ = oracle_run(net, [cases[1]])
    post, lp, st, _ = gpu_run(net, cases)
    assert st[0] == fbn.FBN_E_ZERO_EVIDENCE and lp[0] == -np.inf
    check_fp64(post[1:], lp[1:], st[1:], ref1, "neighbour slot")
    post, lp, st, _ = gpu_run(net, cases, precision=fbn.FBN_FP32_RESCALED)
    assert st[0] == fbn.FBN_E_UNDERFLOW and st[1] == 0


def test_slot_reuse_and_non_contiguous_slots():
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)[:10]
    ref, _ = oracle_run(net, cases)
    say("slot reuse")
    jt = fbn.JT(fbn.net_from_spec(net), max_slots=16)
    slots = [15, 3, 9, 0, 7, 12, 1, 5, 11, 2]
    post, lp, st, _ = gpu_run(net, cases, jt=jt, slots=slots)
    check_fp64(post, lp, st, ref, "scattered slots")
    post, lp, st, _ = gpu_run(net, cases[::-1], jt=jt, slots=slots)
    check_fp64(post, lp, st, ref[::-1], "reused slots")
    # clearing evidence
    fbn.set_evidence(jt, 3, [], [])
    lp0, st0 = fbn.calibrate(jt, [3], want_results=True)
    assert st0[0] == 0 and abs(lp0[0]) < 1e-12


def test_batched_equals_alone():
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:12]
    say("batched == alone")
    post_b, lp_b, _, _ = gpu_run(net, cases)
    jt = fbn.JT(fbn.net_from_spec(net), max_slots=1)
    for k in (0, 5, 11):
        post_a, lp_a, _, _ = gpu_run(net, [cases[k]], jt=jt)
        assert np.max(np.abs(post_a[0] - post_b[k])) <= 1e-12 * np.max(post_b[k])
        assert abs(lp_a[0] - lp_b[k]) <= 1e-12 * abs(lp_b[k])


def test_query_marginals_subset_and_errors():
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)[:2]
    say("query subset")
    post, lp, st, jt = gpu_run(net, cases)
    offs = np.concatenate([[0], np.cumsum(net.card)])
    vs = [5, 0, 23]
    got = fbn.query_marginals(jt, 1, vs, net.card)
    want = np.concatenate([post[1][offs[v]:offs[v + 1]] for v in vs])
    assert np.array_equal(got, want)
    with pytest.raises(fbn.FbnError):
        fbn.set_evidence(jt, 0, [0, 0], [0, 1])
    with pytest.raises(fbn.FbnError):
        fbn.set_evidence(jt, 0, [0], [9])
    with pytest.raises(fbn.FbnError):
        fbn.calibrate(jt, [0, 0])
    with pytest.raises(fbn.FbnError):
        fbn.calibrate(jt, [2])


@pytest.mark.parametrize("prec", [fbn.FBN_FP64, fbn.FBN_FP32_RESCALED])
def test_graph_replay_equals_eager(prec):
    # the captured layer sequence, replayed several times with new evidence,
    # eager work and synchronisation in between, gives bitwise the eager result
    import torch
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:24]
    say("graph replay", prec)
    marg = int(np.sum(net.card))
    eager = fbn.JT(fbn.net_from_spec(net), precision=prec, max_slots=8)
    s = torch.cuda.Stream()
    graph = fbn.JT(fbn.net_from_spec(net), precision=prec, max_slots=8, stream=s.cuda_stream)
    fbn.set_graph_mode(graph, True)
    slots = list(range(8))
    for rep in range(3):
        batch = cases[8 * rep: 8 * rep + 8]
        fbn.set_evidence_batch(eager, slots, batch)
        fbn.set_evidence_batch(graph, slots, batch)
        fbn.calibrate(eager, slots)
        pe, le, se = fbn.query_all(eager, slots, marg)
        fbn.calibrate(graph, slots)
        pg, lg, sg = fbn.query_all(graph, slots, marg)
        torch.cuda.synchronize()
        assert np.array_equal(pe, pg) and np.array_equal(le, lg) and np.array_equal(se, sg), rep
        # a different batch size captures its own graph
        fbn.set_evidence(graph, 0, *cases[rep])
        fbn.set_evidence(eager, 0, *cases[rep])
        lg1, _ = fbn.calibrate(graph, [0], want_results=True)
        le1, _ = fbn.calibrate(eager, [0], want_results=True)
        assert np.array_equal(lg1, le1)
    ref, _ = oracle_run(net, cases[16:24])
    (check_fp64 if prec == fbn.FBN_FP64 else check_fp32)(pg, lg, sg, ref, "graph")
    del graph
    torch.cuda.synchronize()


def test_torch_stream_and_allocator():
    import torch
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)[:8]
    say("torch stream + allocator")
    ref, _ = oracle_run(net, cases)
    s = torch.cuda.Stream()
    jt = fbn.JT(fbn.net_from_spec(net), max_slots=8, stream=s.cuda_stream, torch_allocator=True)
    post, lp, st, _ = gpu_run(net, cases, jt=jt)
    check_fp64(post, lp, st, ref, "torch")
    del jt
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,tile", [(fbn.FBN_FP32_RESCALED, 512), (fbn.FBN_FP64, 256), (fbn.FBN_FP32_RESCALED, 100)])
def test_eight_slots_per_workgroup(prec, tile):
    # small tiles let one workgroup carry eight slots; ragged batch sizes
    # leave some of a workgroup's slots empty
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:19]
    say("eight slots per workgroup", prec, tile)
    ref, _ = oracle_run(net, cases)
    post, lp, st, jt = gpu_run(net, cases, precision=prec, tile=tile)
    (check_fp64 if prec == fbn.FBN_FP64 else check_fp32)(post, lp, st, ref, f"B8 tile {tile}")
    # the same case alone in the same tree: bitwise equal
    marg = int(np.sum(net.card))
    fbn.set_evidence(jt, 18, *cases[3])
    lp1, _ = fbn.calibrate(jt, [18], want_results=True)
    p1, _, _ = fbn.query_all(jt, [18], marg)
    assert np.array_equal(p1[0], post[3]) and lp1[0] == lp[3]

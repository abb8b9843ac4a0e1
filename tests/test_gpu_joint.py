"""GPU parity of joint posteriors P(Q | e) for query variables sharing a
clique (the paper's problem statement asks for the conditional probability
of the query variables given the evidence, Section 1), through the C ABI,
against the FP64 oracle's joint query on the same seeded inputs.  Bars as
for single-variable posteriors: FP64 within 1e-12 relative per entry (oracle
zeros exact), FP32 within 1e-5 absolute."""
import numpy as np
import pytest

import fbngen
import oracle
from paper_2212_04241_amd import fbn
from tests.gpu_util import FP32_ATOL, FP64_RTOL, say

pytestmark = pytest.mark.gpu


def _query_sets(ojt, rng, k):
    """k query sets: random subsets (sizes 1..3) of random cliques, plus the
    whole of the smallest and of the largest clique."""
    sizes = [ojt.clique_size(c) for c in range(ojt.n_cliques)]
    out = []
    for _ in range(k):
        c = int(rng.integers(0, ojt.n_cliques))
        vs, _, _ = ojt.clique(c)
        m = int(rng.integers(1, min(3, len(vs)) + 1))
        out.append([int(x) for x in rng.permutation(vs)[:m]])
    out.append([int(x) for x in ojt.clique(int(np.argmin(sizes)))[0]])
    big = [int(x) for x in ojt.clique(int(np.argmax(sizes)))[0]]
    out.append(big[:1])
    out.append(big[-2:][::-1])
    return out


def _check(got, want, fp32, label):
    assert got.shape == want.shape, label
    if fp32:
        err = float(np.max(np.abs(got - want)))
        assert err <= FP32_ATOL, (label, err)
        return err
    bad = np.abs(got - want) > FP64_RTOL * np.abs(want) + 1e-300
    assert not bad.any(), (label, float(np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300))))
    return 0.0


def _run(net, cases, qsets, precision, layout, tile=0):
    ojt = oracle.compile_net(net)
    n = len(cases)
    jt = fbn.JT(fbn.net_from_spec(net), precision=precision, max_slots=n, layout=layout, tile_entries=tile)
    slots = list(range(n))
    fbn.set_evidence_batch(jt, slots, cases)
    _, st = fbn.calibrate(jt, slots, want_results=True)
    assert not st.any()
    worst = 0.0
    for k, (v, s) in enumerate(cases):
        for q in qsets:
            want = oracle.query_joint(ojt, v, s, q)
            got = fbn.query_joint(jt, k, q, net.card)
            worst = max(worst, _check(got, want, precision == fbn.FBN_FP32_RESCALED, (k, q)))
    jt.free()
    return worst


@pytest.mark.parametrize("precision", [fbn.FBN_FP64, fbn.FBN_FP32_RESCALED])
@pytest.mark.parametrize("layout", [fbn.FBN_LAYOUT_PER_SLOT, fbn.FBN_LAYOUT_INTERLEAVED])
def test_joint_c1(precision, layout):
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)[:12]
    qsets = _query_sets(oracle.compile_net(net), np.random.default_rng(1), 8)
    say("joint C1", precision, layout, len(qsets))
    say("worst", _run(net, cases, qsets, precision, layout))


@pytest.mark.parametrize("precision", [fbn.FBN_FP64, fbn.FBN_FP32_RESCALED])
@pytest.mark.parametrize("layout", [fbn.FBN_LAYOUT_PER_SLOT, fbn.FBN_LAYOUT_INTERLEAVED])
def test_joint_c2_large_cliques(precision, layout):
    # C2's largest cliques (3^10 entries) split each output over many chunks
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:3]
    qsets = _query_sets(oracle.compile_net(net), np.random.default_rng(2), 4)
    say("joint C2", precision, layout, qsets)
    say("worst", _run(net, cases, qsets, precision, layout))


def test_joint_c3_huge_clique_fp32():
    net = fbngen.make_net("C3", 0)
    cases = fbngen.make_cases("C3", net)[:1]
    ojt = oracle.compile_net(net)
    sizes = [ojt.clique_size(c) for c in range(ojt.n_cliques)]
    big = [int(x) for x in ojt.clique(int(np.argmax(sizes)))[0]]
    qsets = [big[:1], big[:2], [big[-1], big[0]]]
    say("joint C3", max(sizes), qsets)
    say("worst", _run(net, cases, qsets, fbn.FBN_FP32_RESCALED, fbn.FBN_LAYOUT_INTERLEAVED))


def test_single_variable_joint_equals_posterior():
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)[:4]
    jt = fbn.JT(fbn.net_from_spec(net), max_slots=4)
    fbn.set_evidence_batch(jt, range(4), cases)
    fbn.calibrate(jt, range(4))
    post, _, st = fbn.query_all(jt, range(4), int(np.sum(net.card)))
    off = np.concatenate([[0], np.cumsum(net.card)])
    for k in range(4):
        for v in range(net.n):
            got = fbn.query_joint(jt, k, [v], net.card)
            want = post[k, off[v]:off[v + 1]]
            assert np.all(np.abs(got - want) <= 1e-13 * np.abs(want) + 1e-300), (k, v)


def test_joint_order_of_query_variables_transposes():
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)[:1]
    ojt = oracle.compile_net(net)
    c = next(c for c in range(ojt.n_cliques) if len(ojt.clique(c)[0]) >= 2)
    vs = [int(x) for x in ojt.clique(c)[0]][:2]
    jt = fbn.JT(fbn.net_from_spec(net), max_slots=1)
    fbn.set_evidence_batch(jt, [0], cases)
    fbn.calibrate(jt, [0])
    a = fbn.query_joint(jt, 0, vs, net.card).reshape(int(net.card[vs[0]]), int(net.card[vs[1]]))
    b = fbn.query_joint(jt, 0, vs[::-1], net.card).reshape(int(net.card[vs[1]]), int(net.card[vs[0]]))
    assert np.array_equal(a, b.T)


def test_joint_errors():
    net = fbngen.make_net("C1", 0)
    ojt = oracle.compile_net(net)
    jt = fbn.JT(fbn.net_from_spec(net), max_slots=1)
    fbn.set_evidence(jt, 0, [], [])
    fbn.calibrate(jt, [0])
    # a pair of variables that share no clique
    together = set()
    for c in range(ojt.n_cliques):
        vs = [int(x) for x in ojt.clique(c)[0]]
        together |= {(a, b) for a in vs for b in vs}
    apart = next((a, b) for a in range(net.n) for b in range(net.n) if a != b and (a, b) not in together)
    for q in ([], [0, 0], [net.n], list(apart)):
        with pytest.raises(fbn.FbnError) as ei:
            fbn.query_joint(jt, 0, q, np.append(net.card, 2))
        assert ei.value.code == fbn.FBN_E_INVALID_ARG, q
    with pytest.raises(fbn.FbnError) as ei:
        fbn.query_joint(jt, 1, [0], net.card)
    assert ei.value.code == fbn.FBN_E_INVALID_ARG


def test_joint_zero_evidence_slot():
    text = ("fbn 1\nvars 3\nvar 0 2 0\nvar 1 2 1 0\nvar 2 2 1 1\ncpt 0 2\n1 0\ncpt 1 4\n1 0 0.5 0.5\n"
            "cpt 2 4\n0.5 0.5 0.25 0.75\nend\n")
    net = fbngen.net_from_text(text)
    for prec, code in ((fbn.FBN_FP64, fbn.FBN_E_ZERO_EVIDENCE), (fbn.FBN_FP32_RESCALED, fbn.FBN_E_UNDERFLOW)):
        jt = fbn.JT(fbn.net_from_spec(net), precision=prec, max_slots=2)
        fbn.set_evidence_batch(jt, [0, 1], [([1], [1]), ([2], [1])])
        fbn.calibrate(jt, [0, 1])
        with pytest.raises(fbn.FbnError) as ei:
            fbn.query_joint(jt, 0, [0, 1], net.card)
        assert ei.value.code == code
        ojt = oracle.compile_net(net)
        got = fbn.query_joint(jt, 1, [1, 2], net.card)
        want = oracle.query_joint(ojt, [2], [1], [1, 2])
        _check(got, want, prec == fbn.FBN_FP32_RESCALED, "neighbour slot")
        jt.free()

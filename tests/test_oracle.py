"""Pins of the FP64 oracle against facts that do not come from the oracle.

The paper (a two-page poster) prints no worked example, posterior or P(e); it
poses exact inference as the conditional probability of query variables given
evidence (Section 1).  So the oracle is pinned by that definition evaluated by
other means: hand-derived exact fractions, brute-force enumeration of the
joint, forward-backward smoothing on chains, the naive-Bayes closed form, and
structural facts of junction trees checked with networkx.
"""
import itertools
import json
import os
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import fbngen
import oracle
from tests import refmath

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "micro")


def _read(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return f.read()


# ---------------------------------------------------------------- golden

def test_micro_nets_exact_fractions():
    with open(os.path.join(GOLDEN, "expected.json")) as f:
        spec = json.load(f)
    for case in spec["cases"]:
        text = _read(case["net"])
        jt = oracle.OracleJT(oracle.OracleNet.from_text(text))
        ev = case["evidence"]
        lp, post = jt.query([v for v, _ in ev], [s for _, s in ev])
        pe = float(Fraction(case["pe"]))
        assert abs(np.exp(lp) - pe) <= 1e-15 * pe, case
        want = np.array([float(Fraction(x)) for row in case["post"] for x in row])
        assert np.max(np.abs(post - want)) <= 1e-15, (case, post, want)


def test_micro_nets_match_brute_force_too():
    # the golden fractions and the enumerator agree, so neither is mistyped
    with open(os.path.join(GOLDEN, "expected.json")) as f:
        spec = json.load(f)
    for case in spec["cases"]:
        net = fbngen.net_from_text(_read(case["net"]))
        ev = case["evidence"]
        pe, post = refmath.brute_force(net, [v for v, _ in ev], [s for _, s in ev])
        assert abs(pe - float(Fraction(case["pe"]))) < 1e-15
        want = np.array([float(Fraction(x)) for row in case["post"] for x in row])
        assert np.max(np.abs(post - want)) < 1e-15


def test_hex_floats_round_trip_exactly():
    net = fbngen.random_small_net(7, 6)
    jt_text = oracle.OracleJT(oracle.OracleNet.from_text(net.to_text()))
    jt_arr = oracle.compile_net(net)
    assert np.array_equal(jt_text.prior(), jt_arr.prior())


# ---------------------------------------------------------------- brute force

def _check_against_brute(net, vars_, states, rtol=1e-13):
    jt = oracle.compile_net(net)
    lp, post = jt.query(vars_, states)
    pe, want = refmath.brute_force(net, vars_, states)
    assert abs(np.exp(lp) - pe) <= rtol * pe
    assert np.all(np.abs(post - want) <= rtol * np.maximum(want, 1e-300) + 1e-300) or \
        np.max(np.abs(post - want)) <= 1e-14


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 11), max_card=st.integers(2, 3),
       p_max=st.integers(0, 3), frac=st.floats(0.0, 0.6))
def test_posteriors_match_brute_force(seed, n, max_card, p_max, frac):
    net = fbngen.random_small_net(seed, n, max_card=max_card, p_max=p_max)
    rng = np.random.default_rng(seed ^ 0x5EED)
    k = int(round(frac * n))
    vs = np.sort(rng.choice(n, size=k, replace=False)) if k else np.zeros(0, dtype=int)
    ss = [int(rng.integers(0, int(net.card[v]))) for v in vs]
    _check_against_brute(net, vs, ss)


@pytest.mark.parametrize("seed", range(6))
def test_windowed_dags_match_brute_force(seed):
    net = fbngen.random_small_net(100 + seed, 13, max_card=3, p_max=3, window=4, alpha=0.3)
    rng = np.random.default_rng(seed)
    vs = np.sort(rng.choice(13, size=4, replace=False))
    ss = [int(rng.integers(0, int(net.card[v]))) for v in vs]
    _check_against_brute(net, vs, ss)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("seed", range(4))
def test_chain_equals_forward_backward(seed):
    rng = np.random.default_rng(seed)
    n = 14
    card = rng.integers(2, 5, size=n).astype(np.int32)
    parents = [[]] + [[t - 1] for t in range(1, n)]
    prior0 = rng.dirichlet(np.ones(card[0]))
    trans = [rng.dirichlet(np.ones(card[t + 1]), size=card[t]) for t in range(n - 1)]
    cpt = [prior0] + [trans[t].ravel() for t in range(n - 1)]
    net = fbngen.Net(card, parents, cpt)
    obs = {2: 1, 7: 0, 13: 1}
    jt = oracle.compile_net(net)
    lp, post = jt.query(list(obs.keys()), list(obs.values()))
    pe, fb = refmath.chain_forward_backward(prior0, trans, obs)
    assert abs(np.exp(lp) - pe) <= 1e-13 * pe
    assert np.max(np.abs(post - np.concatenate(fb))) <= 1e-13


def test_naive_bayes_star_closed_form():
    rng = np.random.default_rng(3)
    nc = 9
    rh = 5
    card = np.array([rh] + list(rng.integers(2, 5, size=nc)), dtype=np.int32)
    prior_h = rng.dirichlet(np.full(rh, 0.5))
    cond = [rng.dirichlet(np.full(card[j + 1], 0.5), size=rh) for j in range(nc)]
    net = fbngen.Net(card, [[]] + [[0]] * nc, [prior_h] + [c.ravel() for c in cond])
    obs = {0: 1, 3: 0, 4: 1, 8: 1}
    jt = oracle.compile_net(net)
    lp, post = jt.query([j + 1 for j in obs], list(obs.values()))
    pe, ph, pc = refmath.naive_bayes(prior_h, cond, obs)
    want = np.concatenate([ph] + [pc[j] for j in range(nc)])
    assert abs(np.exp(lp) - pe) <= 1e-13 * pe
    assert np.max(np.abs(post - want)) <= 1e-13


def test_no_evidence_root_variable_is_its_cpt():
    net = fbngen.random_small_net(11, 9)
    jt = oracle.compile_net(net)
    lp, post = jt.query([], [])
    assert abs(lp) < 1e-14
    offs = np.concatenate([[0], np.cumsum(net.card)])
    for v in range(net.n):
        if not net.parents[v]:
            assert np.max(np.abs(post[offs[v]:offs[v + 1]] - net.cpt[v])) < 1e-14


def test_evidence_on_roots_only_gives_product_of_priors():
    net = fbngen.random_small_net(12, 10)
    roots = [v for v in range(net.n) if not net.parents[v]]
    states = [int(net.card[v]) - 1 for v in roots]
    jt = oracle.compile_net(net)
    lp, _ = jt.query(roots, states)
    want = np.prod([net.cpt[v][s] for v, s in zip(roots, states)])
    assert abs(np.exp(lp) - want) <= 1e-13 * want


def test_d_separated_evidence_leaves_posterior_unchanged():
    # two disconnected chains: evidence on one leaves the other's posteriors
    rng = np.random.default_rng(5)
    card = np.array([2, 3, 2, 3, 2, 2], dtype=np.int32)
    parents = [[], [0], [1], [], [3], [4]]
    cpt = [rng.dirichlet(np.ones(card[v]), size=int(np.prod([card[p] for p in parents[v]] or [1]))).ravel()
           for v in range(6)]
    net = fbngen.Net(card, parents, cpt)
    jt = oracle.compile_net(net)
    _, p0 = jt.query([], [])
    _, p1 = jt.query([5], [1])
    assert np.max(np.abs(p0[:7] - p1[:7])) < 1e-14


# ---------------------------------------------------------------- invariants

def _layout(jt, c):
    vs, _, _ = jt.clique(c)
    return [int(v) for v in vs]


def _calibrated(jt, vars_, states):
    lp, post, tab, sep = jt.query(vars_, states, tables=True, seps=True)
    tables, o = [], 0
    for c in range(jt.n_cliques):
        m = jt.clique_size(c)
        tables.append(tab[o:o + m]); o += m
    seps, o = [], 0
    for e in range(jt.n_edges):
        m = int(np.prod([int(jt.card[v]) for v in jt.edge(e)[2]], dtype=np.int64))
        seps.append(sep[o:o + m]); o += m
    return lp, post, tables, seps


def _marginal(table, layout, card, target):
    """Marginal of a clique table onto the variables `target`, laid out in
    the order given (last fastest)."""
    keep = set(target)
    t = np.asarray(table).reshape([int(card[v]) for v in layout]) if layout else np.asarray(table).reshape(())
    axes = tuple(i for i, v in enumerate(layout) if v not in keep)
    m = t.sum(axis=axes)
    kept = [v for v in layout if v in keep]
    order = [kept.index(v) for v in target]
    return np.transpose(m, order).ravel() if kept else np.atleast_1d(m)


@pytest.mark.parametrize("seed", range(5))
def test_calibration_invariants_medium_nets(seed):
    # beyond brute force: n = 40, windowed parents
    net = fbngen.random_small_net(200 + seed, 40, max_card=3, p_max=2, window=8, alpha=0.5)
    rng = np.random.default_rng(seed)
    vs = np.sort(rng.choice(40, size=6, replace=False))
    ss = [int(rng.integers(0, int(net.card[v]))) for v in vs]
    jt = oracle.compile_net(net)
    lp, post, tables, seps = _calibrated(jt, vs, ss)
    pe = np.exp(lp)
    for c in range(jt.n_cliques):
        assert abs(tables[c].sum() - pe) <= 1e-12 * pe
    for e in range(jt.n_edges):
        p, ch, sv = jt.edge(e)
        target = [int(v) for v in sv]
        mp = _marginal(tables[p], _layout(jt, p), jt.card, target)
        mc = _marginal(tables[ch], _layout(jt, ch), jt.card, target)
        scale = max(np.max(np.abs(seps[e])), 1e-300)
        assert np.max(np.abs(mp - seps[e])) <= 1e-12 * scale
        assert np.max(np.abs(mc - seps[e])) <= 1e-12 * scale
    offs = np.concatenate([[0], np.cumsum(net.card)])
    for v in range(net.n):
        assert abs(post[offs[v]:offs[v + 1]].sum() - 1.0) < 1e-13


@pytest.mark.parametrize("seed", range(4))
def test_factorisation_equals_joint_times_evidence(seed):
    net = fbngen.random_small_net(300 + seed, 7, max_card=3, p_max=3)
    vs, ss = [1, 4], [1, 0]
    jt = oracle.compile_net(net)
    _, _, tables, seps = _calibrated(jt, vs, ss)
    prior = jt.prior()
    P = refmath.joint(net)
    layouts = [_layout(jt, c) for c in range(jt.n_cliques)]
    offs = np.concatenate([[0], np.cumsum([jt.clique_size(c) for c in range(jt.n_cliques)])])
    for x in itertools.product(*[range(int(r)) for r in net.card]):
        num = 1.0
        pri = 1.0
        for c in range(jt.n_cliques):
            lay = layouts[c]
            i = 0
            for v in lay:
                i = i * int(net.card[v]) + x[v]
            num *= tables[c][i]
            pri *= prior[offs[c] + i]
        den = 1.0
        for e in range(jt.n_edges):
            sv = jt.edge(e)[2]
            i = 0
            for v in sv:
                i = i * int(net.card[v]) + x[v]
            den *= seps[e][i]
        consistent = all(x[v] == s for v, s in zip(vs, ss))
        want = P[x] if consistent else 0.0
        got = num / den if den != 0 else 0.0
        assert abs(got - want) <= 1e-12 * max(P[x], 1e-300), (x, got, want)
        assert abs(pri - P[x]) <= 1e-13 * P[x]


# ---------------------------------------------------------------- structure

def _check_structure(net, jt):
    g = refmath.moral_graph(net)
    cliques = [set(int(v) for v in jt.clique(c)[0]) for c in range(jt.n_cliques)]
    filled = nx.Graph()
    filled.add_nodes_from(range(net.n))
    for C in cliques:
        filled.add_edges_from(itertools.combinations(sorted(C), 2))
    # moral graph is contained in the triangulated graph, which is chordal
    assert all(filled.has_edge(a, b) for a, b in g.edges())
    assert nx.is_chordal(filled)
    # the elimination order is a perfect elimination ordering of it
    order = [int(v) for v in jt.elim_order()]
    assert sorted(order) == list(range(net.n))
    pos = {v: i for i, v in enumerate(order)}
    for v in order:
        later = [u for u in filled.neighbors(v) if pos[u] > pos[v]]
        assert all(filled.has_edge(a, b) for a, b in itertools.combinations(later, 2))
    # the cliques are exactly the maximal cliques of the triangulated graph
    assert set(map(frozenset, cliques)) == set(map(frozenset, nx.find_cliques(filled)))
    assert len(cliques) == len(set(map(frozenset, cliques)))
    # every family lies in some clique; its CPT home is the smallest such
    size = [jt.clique_size(c) for c in range(jt.n_cliques)]
    cpt_home, var_home = jt.homes()
    for v in range(net.n):
        fam = set([v] + list(net.parents[v]))
        ok = [c for c in range(jt.n_cliques) if fam <= cliques[c]]
        assert ok and cpt_home[v] == min(ok, key=lambda c: (size[c], c))
        okv = [c for c in range(jt.n_cliques) if v in cliques[c]]
        assert var_home[v] == min(okv, key=lambda c: (size[c], c))
    # a spanning tree with maximum total separator size
    t = nx.Graph()
    t.add_nodes_from(range(jt.n_cliques))
    for e in range(jt.n_edges):
        p, ch, sv = jt.edge(e)
        assert set(int(v) for v in sv) == cliques[p] & cliques[ch]
        # a separator's variables keep the order they take in the parent's layout
        player = [int(v) for v in jt.clique(p)[0]]
        assert [int(v) for v in sv] == [v for v in player if v in set(int(x) for x in sv)]
        t.add_edge(p, ch)
    assert jt.n_edges == jt.n_cliques - 1 and nx.is_connected(t)
    full = nx.Graph()
    for i, j in itertools.combinations(range(jt.n_cliques), 2):
        full.add_edge(i, j, weight=len(cliques[i] & cliques[j]))
    if jt.n_cliques > 1:
        best = sum(d["weight"] for _, _, d in nx.maximum_spanning_tree(full).edges(data=True))
        got = sum(len(cliques[p] & cliques[ch]) for p, ch in t.edges())
        assert got == best
    # running intersection
    for i, j in itertools.combinations(range(jt.n_cliques), 2):
        inter = cliques[i] & cliques[j]
        for c in nx.shortest_path(t, i, j):
            assert inter <= cliques[c]
    # root: minimum eccentricity, lowest id on ties; depth and height
    ecc = nx.eccentricity(t) if jt.n_cliques > 1 else {0: 0}
    assert jt.root == min(range(jt.n_cliques), key=lambda c: (ecc[c], c))
    dist = nx.single_source_shortest_path_length(t, jt.root)
    for c in range(jt.n_cliques):
        lay, h, d = jt.clique(c)
        assert d == dist[c]
        kids = [u for u in t.neighbors(c) if dist[u] == d + 1]
        assert h == (0 if not kids else 1 + max(jt.clique(u)[1] for u in kids))
        # layout: root ascending; others [separator asc] ++ [rest asc]
        lay = [int(v) for v in lay]
        if c == jt.root:
            assert lay == sorted(lay)
        else:
            e = [e for e in range(jt.n_edges) if jt.edge(e)[1] == c]
            assert len(e) == 1
            sv = [int(v) for v in jt.edge(e[0])[2]]
            assert lay == sv + sorted(set(lay) - set(sv))
    # edges numbered by ascending child id
    assert [jt.edge(e)[1] for e in range(jt.n_edges)] == sorted(c for c in range(jt.n_cliques) if c != jt.root)
    # index maps re-derived by decoding every parent entry
    for e in range(jt.n_edges):
        p, ch, sv = jt.edge(e)
        lay = [int(v) for v in jt.clique(p)[0]]
        m = jt.index_map(e)
        cards = [int(net.card[v]) for v in lay]
        scards = [int(net.card[v]) for v in sv]
        for j in range(len(m)):
            dg = dict(zip(lay, refmath.digits(j, cards)))
            want = 0
            for v, r in zip(sv, scards):
                want = want * r + dg[int(v)]
            assert m[j] == want


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 16), p_max=st.integers(0, 3))
def test_structure_properties(seed, n, p_max):
    net = fbngen.random_small_net(seed, n, max_card=3, p_max=p_max)
    _check_structure(net, oracle.compile_net(net))


def test_structure_c1_workload():
    net = fbngen.make_net("C1", 0)
    jt = oracle.compile_net(net)
    assert jt.max_clique <= 4096
    _check_structure(net, jt)


def test_minfill_hand_worked_diamond():
    # binary diamond 0->1, 0->2, 1->3, 2->3: moralising joins 1-2.  Vertices 0
    # and 3 need no fill; equal weights, so 0 goes first: clique {0,1,2};
    # then 1 (no fill, lowest id): clique {1,2,3}; {2,3} and {3} are subsumed.
    net = fbngen.net_from_text(_read("diamond.fbn"))
    jt = oracle.compile_net(net)
    assert list(jt.elim_order()) == [0, 1, 2, 3]
    assert [list(jt.clique(c)[0]) for c in range(jt.n_cliques)] == [[0, 1, 2], [1, 2, 3]]
    assert jt.root == 0
    p, ch, sv = jt.edge(0)
    assert (p, ch, list(sv)) == (0, 1, [1, 2])
    assert list(jt.index_map(0)) == [j % 4 for j in range(8)]
    # with variable 0 given 3 states, vertex 3 has the smaller weight and goes
    # first: cliques {1,2,3} (id 0) then {0,1,2} (id 1); root is the lowest id
    net.card = np.array([3, 2, 2, 2], dtype=np.int32)
    net.cpt = [np.array([0.25, 0.25, 0.5]), np.array([0.5, 0.5] * 3), net.cpt[2].tolist() + [0.5, 0.5], net.cpt[3]]
    net.cpt[2] = np.array(net.cpt[2])
    jt = oracle.compile_net(net)
    assert int(jt.elim_order()[0]) == 3
    assert [list(jt.clique(c)[0]) for c in range(jt.n_cliques)] == [[1, 2, 3], [1, 2, 0]]
    assert jt.root == 0


def test_minfill_golden_cycle_with_pendants():
    # a chordless 4-cycle with two pendant-like vertices, derived by hand in
    # tests/golden/minfill/expected.json: min-fill, min-weight and min-fill
    # without the weight term choose different first vertices, and the chord
    # of the cycle is placed by the id tie-break
    gdir = os.path.join(os.path.dirname(__file__), "golden", "minfill")
    with open(os.path.join(gdir, "expected.json")) as f:
        want = json.load(f)
    with open(os.path.join(gdir, want["net"])) as f:
        net = fbngen.net_from_text(f.read())
    jt = oracle.compile_net(net)
    assert [int(x) for x in jt.elim_order()] == want["elim_order"]
    assert [[int(x) for x in jt.clique(c)[0]] for c in range(jt.n_cliques)] == want["cliques"]
    assert jt.root == want["root"]
    assert [jt.clique(c)[1] for c in range(jt.n_cliques)] == want["height"]
    assert [jt.clique(c)[2] for c in range(jt.n_cliques)] == want["depth"]
    for e, (p, ch, sv) in enumerate(want["edges"]):
        gp, gc, gs = jt.edge(e)
        assert (gp, gc, [int(x) for x in gs]) == (p, ch, sv)
        assert [int(x) for x in jt.index_map(e)] == want["maps"][e]
    ch, vh = jt.homes()
    assert [int(x) for x in ch] == want["cpt_home"]
    assert [int(x) for x in vh] == want["var_home"]


def _tiny_mass_net():
    # X (4097 states) -> Y (2) -> Z (2).  P(X=0) = 1 - 2^-48 and each of the
    # other 4096 states has 2^-60, so the stored CPT sums to exactly 1.  In
    # ascending order every 2^-60 (or 2^-61 after halving) is below half an
    # ulp of the running sum and a plain left-to-right sum loses all of them.
    big, tiny = 1.0 - 2.0 ** -48, 2.0 ** -60
    px = np.array([big] + [tiny] * 4096)
    net = fbngen.Net(card=np.array([4097, 2, 2], dtype=np.int32), parents=[[], [0], [1]],
                     cpt=[px, np.full(2 * 4097, 0.5), np.array([0.25, 0.75, 0.5, 0.5])])
    return net, big, tiny


def test_compensated_sums_are_exact_where_plain_summation_is_not():
    # Every table sum of the oracle is compensated (Neumaier 1974), so on this
    # input the collect message onto Y, P(e) and the normaliser of X's
    # posterior are the exact sums of the stored values.
    net, big, tiny = _tiny_mass_net()
    exact = Fraction(big) + 4096 * Fraction(tiny)
    assert exact == 1
    plain = 0.0
    for x in [big] + [tiny] * 4096:
        plain += x
    assert plain == big != 1.0          # what an uncompensated sum returns
    jt = oracle.compile_net(net)
    lp, post = jt.query([], [])
    assert lp == 0.0                    # log of the exact P(e) = 1
    assert post[0] == big and np.all(post[1:4097] == tiny)
    # observing Z = 1: P(e) = sum_y P(y) P(Z=1|y) with P(y) = 1/2 exactly
    lp, post = jt.query([2], [1])
    assert abs(lp - float(np.log(0.625))) <= 2e-16     # uncompensated: off by 3.6e-15
    assert post[0] == big


# ---------------------------------------------------------------- joint queries

def test_joint_posteriors_diamond_exact_fractions():
    # P(A,B,C,D=1) of the diamond in 512ths (tests/golden/micro/expected.json,
    # derived by hand from the joint): A0: 000:12 001:24 010:16 011:28; A1:
    # 100:1 101:14 110:12 111:147, bits A,B,C; total 254.  Summing over A gives
    # P(B,C | D=1) = (13, 38, 28, 175)/254; over C, P(A,B | D=1) = (36, 44, 15, 159)/254.
    net = fbngen.net_from_text(_read("diamond.fbn"))
    jt = oracle.compile_net(net)
    cases = {(1, 2): [13, 38, 28, 175], (2, 1): [13, 28, 38, 175], (0, 1): [36, 44, 15, 159],
             (3, 2, 1): [0, 0, 0, 0, 13, 28, 38, 175]}
    for q, num in cases.items():
        got = oracle.query_joint(jt, [3], [1], list(q))
        want = np.array([float(Fraction(x, 254)) for x in num])
        assert np.max(np.abs(got - want)) <= 1e-15, (q, got, want)
    # without evidence, P(A,B) = P(A) P(B|A) from the CPTs
    got = oracle.query_joint(jt, [], [], [0, 1])
    assert np.max(np.abs(got - np.array([0.375, 0.125, 0.125, 0.375]))) <= 1e-16


def test_joint_errors():
    net = fbngen.net_from_text(_read("diamond.fbn"))
    jt = oracle.compile_net(net)
    for q in ([0, 3], [1, 1], []):        # no common clique, repeated, empty
        with pytest.raises(oracle.OracleError) as ei:
            oracle.query_joint(jt, [], [], q)
        assert ei.value.code == oracle.E_INVALID


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(2, 10), pick=st.integers(0, 10**6))
def test_joint_posteriors_match_brute_force(seed, n, pick):
    net = fbngen.random_small_net(seed, n, max_card=3, p_max=3)
    jt = oracle.compile_net(net)
    rng = np.random.default_rng(pick)
    c = int(rng.integers(0, jt.n_cliques))
    cv = jt.clique(c)[0]
    q = [int(x) for x in rng.permutation(cv)[: int(rng.integers(1, len(cv) + 1))]]
    m = int(rng.integers(0, max(1, n // 3) + 1))
    obs = [int(x) for x in rng.choice(n, size=m, replace=False)]
    states = [int(rng.integers(0, int(net.card[v]))) for v in obs]
    pe, _ = refmath.brute_force(net, obs, states)
    if pe <= 0:
        return
    got = oracle.query_joint(jt, obs, states, q)
    want = refmath.brute_force_joint(net, obs, states, q)
    assert np.max(np.abs(got - want)) <= 1e-13, (q, obs)


@pytest.mark.parametrize("seed", range(3))
def test_joint_marginals_are_the_posteriors(seed):
    # the marginal of a joint onto one member equals that member's posterior
    net = fbngen.random_small_net(700 + seed, 30, max_card=4, p_max=3, window=6)
    jt = oracle.compile_net(net)
    rng = np.random.default_rng(seed)
    obs = [int(x) for x in rng.choice(net.n, size=4, replace=False)]
    states = [int(rng.integers(0, int(net.card[v]))) for v in obs]
    _, post = jt.query(obs, states)
    off = np.concatenate([[0], np.cumsum(net.card)])
    for c in range(jt.n_cliques):
        q = [int(x) for x in jt.clique(c)[0]][:3]
        j = oracle.query_joint(jt, obs, states, q).reshape([int(net.card[v]) for v in q])
        for a, v in enumerate(q):
            m = j.sum(axis=tuple(b for b in range(len(q)) if b != a))
            assert np.max(np.abs(m - post[off[v]:off[v + 1]])) <= 1e-13, (c, v)


# ---------------------------------------------------------------- errors

@pytest.mark.parametrize("text,code", [
    ("fbn 1\nvars 2\nvar 0 2 1 1\nvar 1 2 1 0\ncpt 0 4\n.5 .5 .5 .5\ncpt 1 4\n.5 .5 .5 .5\nend\n", oracle.E_INVALID),
    ("fbn 1\nvars 1\nvar 0 1 0\ncpt 0 1\n1\nend\n", oracle.E_INVALID),
    ("fbn 1\nvars 1\nvar 0 2 0\ncpt 0 2\n0.5 0.6\nend\n", oracle.E_INVALID),
    ("fbn 1\nvars 1\nvar 0 2 0\ncpt 0 2\n0.5\nend\n", oracle.E_PARSE),
    ("fbn 2\nvars 1\n", oracle.E_PARSE),
    ("fbn 1\nvars 1\nvar 0 2 0\ncpt 0 2\n0.5 0.5\n", oracle.E_PARSE),
])
def test_parse_errors(text, code):
    with pytest.raises(oracle.OracleError) as ei:
        oracle.OracleNet.from_text(text)
    assert ei.value.code == code


def test_zero_probability_evidence_is_reported():
    text = "fbn 1\nvars 2\nvar 0 2 0\nvar 1 2 1 0\ncpt 0 2\n1 0\ncpt 1 4\n1 0 0.5 0.5\nend\n"
    jt = oracle.OracleJT(oracle.OracleNet.from_text(text))
    with pytest.raises(oracle.OracleError) as ei:
        jt.query([1], [1])
    assert ei.value.code == oracle.E_ZERO_EVIDENCE


def test_bad_evidence_rejected():
    jt = oracle.compile_net(fbngen.random_small_net(1, 4))
    for vs, ss in [([0, 0], [0, 0]), ([9], [0]), ([0], [7])]:
        with pytest.raises(oracle.OracleError):
            jt.query(vs, ss)

"""CPU tests of the library's host side (no GPU needed).

The junction tree the library compiles (cliques, layouts, edges,
separators, root, layers, homes) and every index map must equal the
oracle's bit for bit on the same network: the structure is a deterministic
function of the network under the fixed tie-breaks of both implementations,
and the two share no code.
"""
import ctypes
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import fbngen
import oracle
from paper_2212_04241_amd import fbn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _host_jt(net, **kw):
    return fbn.JT(fbn.net_from_spec(net), host_only=True, **kw)


def compare_structure(net, ojt, ljt, maps="all"):
    s = ljt.stats
    assert (s["n_cliques"], s["n_edges"], s["root"], s["H"], s["D"]) == \
        (ojt.n_cliques, ojt.n_edges, ojt.root, ojt.H, ojt.D)
    assert (s["T"], s["K"], s["max_clique"]) == (ojt.T, ojt.K, ojt.max_clique)
    assert np.array_equal(fbn.jt_elim_order(ljt), ojt.elim_order())
    for c in range(ojt.n_cliques):
        lv, lh, ld = fbn.jt_clique(ljt, c)
        ov, oh, od = ojt.clique(c)
        assert np.array_equal(lv, ov) and (lh, ld) == (oh, od), c
    la, lb = fbn.jt_homes(ljt)
    oa, ob = ojt.homes()
    assert np.array_equal(la, oa) and np.array_equal(lb, ob)
    edges = range(ojt.n_edges) if maps == "all" else maps
    for e in range(ojt.n_edges):
        lp, lc, ls = fbn.jt_edge(ljt, e)
        op, oc, os_ = ojt.edge(e)
        assert (lp, lc) == (op, oc) and np.array_equal(ls, os_), e
    for e in edges:
        assert np.array_equal(fbn.jt_index_map(ljt, e, net.card), ojt.index_map(e)), e


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 40), max_card=st.integers(2, 5),
       p_max=st.integers(0, 4), window=st.sampled_from([None, 3, 8]))
def test_structure_and_maps_bit_exact_random(seed, n, max_card, p_max, window):
    net = fbngen.random_small_net(seed, n, max_card=max_card, p_max=p_max, window=window)
    try:
        ojt = oracle.compile_net(net, max_entries=1 << 22)
    except oracle.OracleError:
        with pytest.raises(fbn.FbnError):
            _host_jt(net, max_clique_entries=1 << 22)
        return
    compare_structure(net, ojt, _host_jt(net, max_clique_entries=1 << 22))


@pytest.mark.parametrize("key", ["C1", "C2"])
def test_structure_and_maps_bit_exact_workloads(key):
    net = fbngen.make_net(key, 0)
    compare_structure(net, oracle.compile_net(net), _host_jt(net))


def test_structure_bit_exact_hub_workload():
    # the ~10^7-entry clique network: structure in full, maps of a few edges
    net = fbngen.make_net("C3", 0, with_cpts=False)
    ojt = oracle.compile_net(net, structure_only=True)
    ljt = _host_jt(fbngen.Net(net.card, net.parents, [np.ones(net.cpt_size(v)) / net.card[v]
                                                      for v in range(net.n)]))
    sizes = [(ojt.clique_size(ojt.edge(e)[0]), e) for e in range(ojt.n_edges)]
    pick = [e for _, e in sorted(sizes)[:6]] + [max(sizes)[1]]
    compare_structure(net, ojt, ljt, maps=pick)


def test_text_and_arrays_give_same_tree():
    net = fbngen.random_small_net(5, 12, max_card=4)
    a = fbn.JT(fbn.load_net_mem(net.to_text()), host_only=True)
    b = _host_jt(net)
    for c in range(a.stats["n_cliques"]):
        assert np.array_equal(fbn.jt_clique(a, c)[0], fbn.jt_clique(b, c)[0])


# ---------------------------------------------------------------- ABI surface

def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "fbn.h")) as f:
        hdr = f.read()
    names = sorted(set(re.findall(r"\b(fbn_[a-z_0-9]+)\s*\(", hdr)))
    assert "fbn_calibrate" in names and "fbn_build_jt" in names
    L = ctypes.CDLL(fbn.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("text,code", [
    ("fbn 1\nvars 2\nvar 0 2 1 1\nvar 1 2 1 0\ncpt 0 4\n.5 .5 .5 .5\ncpt 1 4\n.5 .5 .5 .5\nend\n", fbn.FBN_E_INVALID_ARG),
    ("fbn 1\nvars 1\nvar 0 1 0\ncpt 0 1\n1\nend\n", fbn.FBN_E_INVALID_ARG),
    ("fbn 1\nvars 1\nvar 0 2 0\ncpt 0 2\n0.5 0.6\nend\n", fbn.FBN_E_INVALID_ARG),
    ("fbn 1\nvars 1\nvar 0 2 0\ncpt 0 2\n0.5\nend\n", fbn.FBN_E_PARSE),
    ("fbn 2\nvars 1\n", fbn.FBN_E_PARSE),
    ("fbn 1\nvars 1\nvar 0 2 0\ncpt 0 2\n0.5 0.5\n", fbn.FBN_E_PARSE),
])
def test_library_rejects_bad_networks(text, code):
    with pytest.raises(fbn.FbnError) as ei:
        fbn.load_net_mem(text)
    assert ei.value.code == code


def test_missing_file_is_io_error():
    with pytest.raises(fbn.FbnError) as ei:
        fbn.load_net("/nonexistent/x.fbn")
    assert ei.value.code == fbn.FBN_E_IO


def test_too_large_clique_rejected():
    net = fbngen.make_net("C1", 0)
    with pytest.raises(fbn.FbnError) as ei:
        _host_jt(net, max_clique_entries=16)
    assert ei.value.code == fbn.FBN_E_TOO_LARGE


def test_host_only_jt_refuses_device_calls():
    jt = _host_jt(fbngen.make_net("C1", 0))
    for call in (lambda: fbn.set_evidence(jt, 0, [0], [0]), lambda: fbn.calibrate(jt, [0])):
        with pytest.raises(fbn.FbnError) as ei:
            call()
        assert ei.value.code == fbn.FBN_E_STATE


def test_bad_options_rejected():
    net = fbn.net_from_spec(fbngen.make_net("C1", 0))
    for kw in ({"max_slots": 0}, {"precision": 7}, {"tile_entries": 1 << 20}):
        with pytest.raises(fbn.FbnError) as ei:
            fbn.JT(net, host_only=True, **kw)
        assert ei.value.code == fbn.FBN_E_INVALID_ARG


@pytest.mark.parametrize("tile", [1, 7, 64, 100, 333, 2048, 4096])
@pytest.mark.parametrize("key", ["C1", "C2"])
def test_plan_bounds_check_passes_for_any_tile(key, tile):
    # the build runs the plan checker (every kernel index bound) and fails
    # with FBN_E_STATE if any bound is violated
    _host_jt(fbngen.make_net(key, 0), tile_entries=tile)


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 30), tile=st.sampled_from([1, 5, 64, 129, 2048]))
def test_plan_bounds_check_random(seed, n, tile):
    net = fbngen.random_small_net(seed, n, max_card=6, p_max=3, window=5)
    _host_jt(net, tile_entries=tile, max_clique_entries=1 << 24)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("key,j", [("C3", 0), ("C5", 7), ("C5", 0)])
def test_plan_bounds_check_large_workloads(key, j, precision):
    # mixes full-segment and partial-sum runs in one layer, and rows near the
    # LDS stage limit; the build runs the plan checker
    net = fbngen.make_net(key, j)
    _host_jt(net, precision=precision)


@pytest.mark.parametrize("tile", [1, 16, 64, 128, 256, 1000])
@pytest.mark.parametrize("key,j", [("C1", 0), ("C2", 0), ("C3", 0), ("C5", 7)])
def test_plan_bounds_check_interleaved(key, j, tile):
    # slot-interleaved plans (finaliser blocks of 16 entries, small
    # separators held in registers, one running maximum per large separator)
    # pass the plan checker for any tile and a batch wider than one wave
    net = fbngen.make_net(key, j)
    jt = _host_jt(net, tile_entries=tile, layout=fbn.FBN_LAYOUT_INTERLEAVED, max_slots=130)
    assert jt.stats["interleaved"] == 1


@pytest.mark.parametrize("key", ["C2", "C3"])
def test_interleaved_slots_hold_no_rebuilt_working_tables(key):
    # the interleaved layout stores psi only for cliques with more than six
    # children: a whole slot then takes less than its T table entries alone
    # would, while a per-slot slot holds all of them
    net = fbngen.make_net(key, 0)
    ps = _host_jt(net, precision=fbn.FBN_FP32_RESCALED, max_slots=64, layout=fbn.FBN_LAYOUT_PER_SLOT).stats
    il = _host_jt(net, precision=fbn.FBN_FP32_RESCALED, max_slots=64, layout=fbn.FBN_LAYOUT_INTERLEAVED).stats
    assert ps["slot_bytes"] > 4 * ps["T"] > il["slot_bytes"]


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 30), tile=st.sampled_from([1, 5, 64, 129, 2048]))
def test_plan_bounds_check_interleaved_random(seed, n, tile):
    net = fbngen.random_small_net(seed, n, max_card=6, p_max=3, window=5)
    _host_jt(net, tile_entries=tile, max_clique_entries=1 << 24, layout=fbn.FBN_LAYOUT_INTERLEAVED)


# ---------------------------------------------------------------- forests

def _forest_parts():
    nets = [fbngen.make_net("C1", 0)]
    nets += [fbngen.random_small_net(seed, n, max_card=4, window=8) for seed, n in ((3, 9), (11, 1), (29, 17))]
    with open(os.path.join(ROOT, "tests", "golden", "micro", "disconnected.fbn")) as f:
        nets.append(fbngen.net_from_text(f.read()))
    return nets


def test_forest_is_the_offset_union_of_the_parts():
    # each network of a forest keeps the tree the oracle compiles for it
    # alone, with variable, clique and edge ids offset by the earlier parts
    nets = _forest_parts()
    ljt = fbn.JT([fbn.net_from_spec(n) for n in nets], host_only=True)
    card = np.concatenate([n.card for n in nets])
    s = ljt.stats
    v0 = c0 = e0 = 0
    H = D = 0
    for net in nets:
        ojt = oracle.compile_net(net)
        assert s["n_trees"] == len(nets)
        for c in range(ojt.n_cliques):
            lv, lh, ld = fbn.jt_clique(ljt, c0 + c)
            ov, oh, od = ojt.clique(c)
            assert np.array_equal(lv, np.asarray(ov) + v0) and (lh, ld) == (oh, od), c
            H, D = max(H, oh), max(D, od)
        for e in range(ojt.n_edges):
            lp, lc, ls = fbn.jt_edge(ljt, e0 + e)
            op, oc, os_ = ojt.edge(e)
            assert (lp, lc) == (op + c0, oc + c0) and np.array_equal(ls, np.asarray(os_) + v0), e
            assert np.array_equal(fbn.jt_index_map(ljt, e0 + e, card), ojt.index_map(e)), e
        v0 += net.n
        c0 += ojt.n_cliques
        e0 += ojt.n_edges
    la, lb = fbn.jt_homes(ljt)
    assert len(la) == v0
    assert (s["n_vars"], s["n_cliques"], s["n_edges"], s["H"], s["D"]) == (v0, c0, e0, H, D)


def test_forest_offsets_and_cases():
    nets = _forest_parts()
    off = fbngen.forest_offsets(nets)
    assert off[0] == 0 and off[-1] == sum(n.n for n in nets)
    cases = [[(np.array([0], np.int32), np.array([1], np.int32))] for _ in nets]
    v, s = fbngen.forest_case(off, cases, 0)
    assert np.array_equal(v, off[:-1]) and np.all(s == 1)


def test_forest_rejects_bad_input():
    with pytest.raises(fbn.FbnError):
        fbn.JT([], host_only=True)
    big = fbngen.make_net("C2", 0, with_cpts=True)
    with pytest.raises(fbn.FbnError) as ei:
        fbn.JT([fbn.net_from_spec(fbngen.make_net("C1", 0)), fbn.net_from_spec(big)], host_only=True,
               max_clique_entries=4096)
    assert ei.value.code == fbn.FBN_E_TOO_LARGE and "network 1" in str(ei.value)


@pytest.mark.parametrize("precision", [fbn.FBN_FP32_RESCALED, fbn.FBN_FP64])
def test_plan_bounds_check_c4_forest(precision):
    # the 256-network batch: its plan passes every kernel bound check at
    # build time (a failing check would raise here)
    nets = [fbngen.make_net("C4", j) for j in range(256)]
    jt = fbn.JT([fbn.net_from_spec(n) for n in nets], host_only=True, precision=precision)
    assert jt.stats["n_trees"] == 256 and jt.stats["n_vars"] == sum(n.n for n in nets)


# ---------------------------------------------------------------- autotuner

def test_tuner_picks_the_fastest_and_caches(tmp_path):
    from paper_2212_04241_amd import tune
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)[:4]
    calls = []

    def fake(nets, cs, precision, max_slots, layout, tile, reps, **kw):
        assert not kw                      # an interleaved winner is not refined
        calls.append((layout, tile))
        if tile == 512:
            raise fbn.FbnError(fbn.FBN_E_INVALID_ARG, "fake")
        if layout == tune.INTERLEAVED and tile == 0:
            return 7.0
        return {0: 5.0, 2048: 3.0, 4096: 4.0, 32: 6.0, 128: 9.0, 256: 2.5}[tile]

    path = str(tmp_path / "tune.json")
    r = tune.tune(net, cases, cache=path, measure=fake)
    assert (r["layout"], r["tile"], r["cached"]) == (tune.INTERLEAVED, 256, False)
    assert len(r["trials"]) == len(tune.DEFAULT_CANDIDATES) - 1
    n = len(calls)
    r2 = tune.tune(net, cases, cache=path, measure=fake)
    assert r2["cached"] and len(calls) == n and (r2["layout"], r2["tile"]) == (r["layout"], r["tile"])
    # another batch size or precision is another key
    tune.tune(net, cases[:2], cache=path, measure=fake)
    assert len(calls) > n
    k1 = tune.network_key(net, 1, 4, 4)
    assert k1 == tune.network_key(net, 1, 4, 4) != tune.network_key(net, 0, 4, 4)


def test_tuner_refines_a_per_slot_choice_one_axis_at_a_time(tmp_path):
    from paper_2212_04241_amd import tune
    net = fbngen.make_net("C1", 0)
    cases = fbngen.make_cases("C1", net)[:8]
    calls = []

    def fake(nets, cs, precision, max_slots, layout, tile, reps, slots_per_block=0, fin_block=0):
        calls.append((layout, tile, slots_per_block, fin_block))
        if layout == tune.INTERLEAVED:
            return 9.0
        base = {0: 5.0, 512: 6.0, 2048: 4.0, 4096: 4.5}[tile]
        # slots per block 2 is 10% faster, 4 only 1% (inside the tolerance);
        # finaliser blocks of 1024 a further 5% on top of the chosen slots
        base *= {0: 1.0, 1: 1.3, 2: 0.9, 4: 0.99}[slots_per_block]
        if fin_block == 1024:
            assert slots_per_block == 2     # refined from the best so far
            base *= 0.95
        return base

    r = tune.tune(net, cases, cache=str(tmp_path / "t.json"), measure=fake)
    assert (r["layout"], r["tile"], r["slots_per_block"], r["fin_block"]) == (tune.PER_SLOT, 2048, 2, 1024)
    assert r["ms"] == pytest.approx(4.0 * 0.9 * 0.95)
    assert [s[:2] for s in r["refine"]] == [["slots_per_block", 1], ["slots_per_block", 2], ["slots_per_block", 4],
                                            ["fin_block", 1024], ["fin_block", 2048]]
    assert all(c[:2] == (tune.PER_SLOT, 2048) for c in calls[len(tune.DEFAULT_CANDIDATES):])
    # cached with its knobs; refine=False is its own key and tries no knob
    n = len(calls)
    assert tune.tune(net, cases, cache=str(tmp_path / "t.json"), measure=fake)["fin_block"] == 1024
    r3 = tune.tune(net, cases, cache=str(tmp_path / "t.json"), measure=fake, refine=False)
    assert len(calls) == n + len(tune.DEFAULT_CANDIDATES) and r3["slots_per_block"] == 0 and r3["refine"] == []


@pytest.mark.parametrize("field,value", [("slots_per_block", 3), ("slots_per_block", 16), ("slots_per_block", -1),
                                         ("fin_block", 32), ("fin_block", 8192), ("fin_block", -4)])
def test_bad_per_slot_knobs_are_rejected(field, value):
    net = fbn.net_from_spec(fbngen.make_net("C1", 0))
    with pytest.raises(fbn.FbnError) as ei:
        fbn.JT(net, host_only=True, **{field: value})
    assert ei.value.code == fbn.FBN_E_INVALID_ARG


def test_finaliser_block_size_reshapes_only_the_finaliser_scratch():
    # C2's large separators are finalised in blocks: smaller blocks mean more
    # of them, so more per-block posterior scratch per slot; the tree and every
    # table are unchanged
    net = fbn.net_from_spec(fbngen.make_net("C2", 0))
    a = fbn.JT(net, host_only=True, precision=fbn.FBN_FP32_RESCALED)
    b = fbn.JT(net, host_only=True, precision=fbn.FBN_FP32_RESCALED, fin_block=256)
    c = fbn.JT(net, host_only=True, precision=fbn.FBN_FP32_RESCALED, slots_per_block=1)
    for k in ("T", "K", "max_clique", "sep_total", "n_cliques"):
        assert a.stats[k] == b.stats[k] == c.stats[k]
    assert b.stats["slot_bytes"] >= a.stats["slot_bytes"] == c.stats["slot_bytes"]

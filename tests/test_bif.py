"""The BIF reader (host, CPU): a hand-written network in BIF and the same
network hand-written in .fbn text load to identical CPTs and compile to
bit-identical junction trees; names, states, defaults, renormalised rows and
malformed files behave as the header documents."""
import os

import numpy as np
import pytest

import fbngen
from paper_2212_04241_amd import fbn

GOLD = os.path.join(os.path.dirname(__file__), "golden", "bif")


def _load(name):
    return fbn.load_net(os.path.join(GOLD, name))


def test_bif_cpts_equal_the_hand_written_fbn():
    a = _load("commute.bif")
    with open(os.path.join(GOLD, "commute.fbn")) as f:
        ref = fbngen.net_from_text(f.read())       # the generator's own parser
    assert fbn.net_n_vars(a) == ref.n == 6
    for v in range(ref.n):
        card, par, cpt = fbn.net_cpt(a, v)
        assert card == int(ref.card[v])
        assert list(par) == [int(p) for p in ref.parents[v]]
        assert np.array_equal(cpt, np.asarray(ref.cpt[v], dtype=np.float64).ravel()), v


def test_bif_names_and_states():
    a = _load("commute.bif")
    names = [fbn.net_var_name(a, v) for v in range(6)]
    assert names == ["weather", "sprinkler", "wet", "slippery", "traffic", "late"]
    assert fbn.net_find_var(a, "traffic") == 4
    assert [fbn.net_state_name(a, 4, s) for s in range(3)] == ["light", "medium", "heavy"]
    assert fbn.net_find_state(a, 0, "rain") == 2
    with pytest.raises(fbn.FbnError):
        fbn.net_find_var(a, "nope")
    with pytest.raises(fbn.FbnError):
        fbn.net_find_state(a, 0, "snow")
    b = _load("commute.fbn")                       # .fbn: ids and indices as names
    assert fbn.net_var_name(b, 5) == "5" and fbn.net_state_name(b, 4, 2) == "2"
    assert fbn.net_find_var(b, "3") == 3


def test_bif_and_fbn_compile_bit_exact():
    trees = []
    for name in ("commute.bif", "commute.fbn"):
        net = _load(name)
        jt = fbn.JT(net, host_only=True)
        card = np.array([fbn.net_cpt(net, v)[0] for v in range(6)])
        t = {"stats": {k: v for k, v in jt.stats.items() if k not in ("device_bytes", "slot_bytes")},
             "elim": fbn.jt_elim_order(jt).tolist(), "homes": [h.tolist() for h in fbn.jt_homes(jt)]}
        t["cliques"] = [(c.tolist(), h, d) for c, h, d in (fbn.jt_clique(jt, k) for k in range(jt.stats["n_cliques"]))]
        t["edges"] = [(p, ch, s.tolist()) for p, ch, s in (fbn.jt_edge(jt, e) for e in range(jt.stats["n_edges"]))]
        t["maps"] = [fbn.jt_index_map(jt, e, card).tolist() for e in range(jt.stats["n_edges"])]
        trees.append(t)
    assert trees[0] == trees[1]
    assert trees[0]["stats"]["n_cliques"] >= 3


def test_bif_renormalises_rounded_rows():
    text = ("variable a { type discrete [ 3 ] { x, y, z }; }\n"
            "probability ( a ) { table 0.333, 0.333, 0.333; }\n")
    net = fbn.load_net_mem(text)
    s = 0.333 + 0.333 + 0.333
    assert np.array_equal(fbn.net_cpt(net, 0)[2], np.array([0.333 / s] * 3))


def test_bif_declarations_may_follow_probabilities_and_names_may_be_quoted():
    text = ('probability ( "b" | a ) { (t) 0.5, 0.5; (f) 0.25, 0.75; }\n'
            "probability ( a ) { table 0.1, 0.9; }\n"
            "variable a { type discrete [ 2 ] { t, f }; }\n"
            'variable "b" { type discrete [ 2 ] { 0, 1 }; }\n')
    net = fbn.load_net_mem(text)
    assert fbn.net_var_name(net, 0) == "a" and fbn.net_var_name(net, 1) == "b"
    assert np.array_equal(fbn.net_cpt(net, 1)[2], np.array([0.5, 0.5, 0.25, 0.75]))


_VARS = ("variable a { type discrete [ 2 ] { t, f }; }\n"
         "variable b { type discrete [ 2 ] { t, f }; }\n")

BAD = [
    (_VARS + "probability ( a ) { table 0.5, 0.5; }\nprobability ( b | a ) { (t) 0.5, 0.5; (u) 0.5, 0.5; }\n",
     fbn.FBN_E_PARSE, "unknown state"),
    (_VARS + "probability ( a ) { table 0.5, 0.5; }\nprobability ( b | a ) { (t) 0.5, 0.5; }\n",
     fbn.FBN_E_PARSE, "no probabilities"),
    (_VARS + "probability ( a ) { table 0.5, 0.5; }\nprobability ( b | c ) { (t) 0.5, 0.5; }\n",
     fbn.FBN_E_PARSE, "undeclared parent"),
    (_VARS + "probability ( a ) { table 0.5, 0.5; }\nprobability ( b | a ) { table 0.5, 0.5, 0.5, 0.5; }\n",
     fbn.FBN_E_PARSE, "ambiguous"),
    (_VARS + "probability ( a ) { table 0.5, 0.5, 0.0; }\nprobability ( b ) { table 0.5, 0.5; }\n",
     fbn.FBN_E_PARSE, "wrong length"),
    (_VARS + "probability ( a ) { table 0.5, 0.4; }\nprobability ( b ) { table 0.5, 0.5; }\n",
     fbn.FBN_E_PARSE, "sums to"),
    (_VARS + "probability ( a | b ) { (t) 0.5, 0.5; (f) 0.5, 0.5; }\n"
     "probability ( b | a ) { (t) 0.5, 0.5; (f) 0.5, 0.5; }\n", fbn.FBN_E_INVALID_ARG, "cycle"),
    (_VARS + "variable a { type discrete [ 2 ] { t, f }; }\n", fbn.FBN_E_PARSE, "declared twice"),
    (_VARS + "probability ( a ) { table 0.5, 0.5; }\n", fbn.FBN_E_PARSE, "no probability block"),
    (_VARS + "/* open", fbn.FBN_E_PARSE, "unterminated comment"),
    ("variable a { type discrete [ 3 ] { t, f }; }\n", fbn.FBN_E_PARSE, "state count"),
    ("variable a { type continuous; }\n", fbn.FBN_E_PARSE, "only discrete"),
    (_VARS + "probability ( a ) { table 0.5, x; }\nprobability ( b ) { table 0.5, 0.5; }\n",
     fbn.FBN_E_PARSE, "bad number"),
]


@pytest.mark.parametrize("text,code,words", BAD)
def test_bif_rejects_malformed(text, code, words):
    with pytest.raises(fbn.FbnError) as ei:
        fbn.load_net_mem(text)
    assert ei.value.code == code
    assert words in str(ei.value), str(ei.value)


def _to_bif(net, rng, names):
    """BIF text of a generated network, written independently of the reader:
    parent rows in a shuffled order, some written through a default row,
    decimal values that read back exactly (shortest round-trip form)."""
    out = ["// written by the test", 'network "t" {', "}"]
    order = rng.permutation(net.n)          # declarations in any order
    for v in order:
        st = ", ".join(f"s{v}_{x}" for x in range(int(net.card[v])))
        out.append(f"variable {names[v]} {{\n  type discrete [ {int(net.card[v])} ] {{ {st} }};\n}}")
    for v in rng.permutation(net.n):
        r = int(net.card[v])
        cpt = np.asarray(net.cpt[v], dtype=np.float64).reshape(-1, r)
        par = net.parents[v]
        if not par:
            out.append(f"probability ( {names[v]} ) {{\n  table " + ", ".join(repr(float(x)) for x in cpt[0]) + ";\n}")
            continue
        lines = [f"probability ( {names[v]} | " + ", ".join(names[p] for p in par) + " ) {"]
        rows = list(range(cpt.shape[0]))
        default_row = rows[int(rng.integers(0, len(rows)))] if len(rows) > 1 and rng.random() < 0.5 else None
        for row in rng.permutation(rows):
            if default_row is not None and np.array_equal(cpt[row], cpt[default_row]) and row != default_row:
                continue
            if row == default_row:
                continue
            digs, x = [], int(row)
            for p in reversed(par):
                digs.append(x % int(net.card[p]))
                x //= int(net.card[p])
            digs = digs[::-1]
            lines.append("  (" + ", ".join(f"s{p}_{d}" for p, d in zip(par, digs)) + ") " +
                         ", ".join(repr(float(y)) for y in cpt[row]) + ";")
        if default_row is not None:
            lines.append("  default " + ", ".join(repr(float(y)) for y in cpt[default_row]) + ";")
        lines.append("}")
        out.append("\n".join(lines))
    return "\n".join(out) + "\n"


@pytest.mark.parametrize("seed", range(12))
def test_bif_round_trip_of_generated_networks(seed):
    net = fbngen.random_small_net(500 + seed, 12, max_card=4, p_max=3, window=5)
    rng = np.random.default_rng(seed)
    names = [f"v{seed}x{v}" for v in range(net.n)]
    text = _to_bif(net, rng, names)
    got = fbn.load_net_mem(text)
    assert fbn.net_n_vars(got) == net.n
    for v in range(net.n):
        k = fbn.net_find_var(got, names[v])
        card, par, cpt = fbn.net_cpt(got, k)
        assert card == int(net.card[v])
        assert [fbn.net_var_name(got, p) for p in par] == [names[p] for p in net.parents[v]]
        assert np.array_equal(cpt, np.asarray(net.cpt[v], dtype=np.float64).ravel()), v

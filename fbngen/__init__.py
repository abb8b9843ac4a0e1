"""Seeded synthetic Bayesian networks and evidence cases.

This module is shared by the oracle side and the GPU side of the tests and the
benchmark.  It draws random structures, cardinalities, CPT values, evidence
cases and arrival times; it holds none of the inference arithmetic (no
triangulation, no junction tree, no propagation).

The paper evaluates on six public bnlearn networks with 2000 random test cases
each observing 20% of the variables (Section 3).  Those networks are not
available here; the five workload shapes below stand in for them, and no
structure or CPT of a public network is reproduced.

Random numbers: every stream is a numpy PCG64 generator whose 64-bit seed is
derived with SplitMix64 (Steele, Lea and Flood, 2014) from (workload k,
network j, stream t, attempt a):
    seed64 = mix(mix(mix(k) ^ j) ^ (t + 16*a))
with streams t = 0 DAG, 1 cardinalities, 2 CPT values, 3 evidence, 4 arrivals.

Which attempt (and, where rejection alone cannot meet a clique-size cap, which
arcs are dropped) is read from ``accepted.json`` next to this file.  That file
is written by ``oracle/select_inputs.py``, which measures clique sizes with the
oracle; this module never computes them.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Net", "seed64", "CONFIGS", "make_net", "make_cases", "make_arrivals",
    "random_dag", "load_accepted", "net_from_text",
]

_M64 = (1 << 64) - 1


def _mix(x: int) -> int:
    """One SplitMix64 output step for state x (adds the golden gamma first)."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def seed64(k: int, j: int, t: int, attempt: int = 0) -> int:
    return _mix(_mix(_mix(k) ^ j) ^ (t + 16 * attempt))


def _rng(k: int, j: int, t: int, attempt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed64(k, j, t, attempt)))


@dataclass
class Net:
    """A discrete Bayesian network.

    card[v]      number of states of variable v (>= 2)
    parents[v]   parent ids of v, in the order the CPT is laid out
    cpt[v]       float64 array, parents in listed order then v fastest
                 (so each row over v's states is contiguous)
    """
    card: np.ndarray
    parents: list
    cpt: list = field(default_factory=list)
    name: str = ""

    @property
    def n(self) -> int:
        return int(len(self.card))

    def cpt_size(self, v: int) -> int:
        s = int(self.card[v])
        for p in self.parents[v]:
            s *= int(self.card[p])
        return s

    # flat arrays for the C entry points of both the oracle and the library
    def flat(self):
        n = self.n
        card = np.ascontiguousarray(self.card, dtype=np.int32)
        npar = np.array([len(p) for p in self.parents], dtype=np.int32)
        par = np.array([q for p in self.parents for q in p], dtype=np.int32)
        if self.cpt:
            cpt = np.concatenate([np.asarray(c, dtype=np.float64).ravel() for c in self.cpt])
        else:
            cpt = np.ones(sum(self.cpt_size(v) for v in range(n)), dtype=np.float64)
        return card, npar, par, np.ascontiguousarray(cpt)

    def to_text(self) -> str:
        """The .fbn text form: header, one line per variable, CPT values as
        C99 hexadecimal floats so that float64 values round-trip exactly."""
        out = [f"fbn 1\nvars {self.n}\n"]
        for v in range(self.n):
            ps = " ".join(str(int(p)) for p in self.parents[v])
            out.append(f"var {v} {int(self.card[v])} {len(self.parents[v])}" + (f" {ps}" if ps else "") + "\n")
        for v in range(self.n):
            vals = np.asarray(self.cpt[v], dtype=np.float64).ravel()
            out.append(f"cpt {v} {vals.size}\n")
            out.append(" ".join(float(x).hex() for x in vals))
            out.append("\n")
        out.append("end\n")
        return "".join(out)


def _num(tok: str) -> float:
    """A CPT value: C99 hexadecimal float ("0x1.8p-2") or plain decimal."""
    t = tok.lower()
    return float.fromhex(tok) if ("0x" in t or "p" in t) else float(tok)


def net_from_text(text: str) -> Net:
    """Parse the .fbn text form (used by tests that write small nets by hand)."""
    toks = text.split()
    pos = 0

    def nxt():
        nonlocal pos
        t = toks[pos]
        pos += 1
        return t

    assert nxt() == "fbn" and nxt() == "1"
    assert nxt() == "vars"
    n = int(nxt())
    card = np.zeros(n, dtype=np.int32)
    parents = [[] for _ in range(n)]
    cpt = [None] * n
    while True:
        t = nxt()
        if t == "end":
            break
        if t == "var":
            v = int(nxt()); card[v] = int(nxt()); k = int(nxt())
            parents[v] = [int(nxt()) for _ in range(k)]
        elif t == "cpt":
            v = int(nxt()); m = int(nxt())
            cpt[v] = np.array([_num(nxt()) for _ in range(m)], dtype=np.float64)
        else:
            raise ValueError(f"bad token {t!r}")
    return Net(card, parents, cpt)


# --------------------------------------------------------------------------
# structure samplers
# --------------------------------------------------------------------------

def random_dag(rng: np.random.Generator, n: int, p_max: int, window: int | None):
    """Parents by topological position: position i draws k ~ U{0..min(p_max,
    #candidates)} and then k distinct parents uniformly among the candidates
    (all earlier positions, or the previous ``window`` ones)."""
    par_pos = []
    for i in range(n):
        lo = 0 if window is None else max(0, i - window)
        cand = np.arange(lo, i)
        k = int(rng.integers(0, min(p_max, cand.size) + 1))
        chosen = rng.choice(cand, size=k, replace=False) if k else np.empty(0, dtype=np.int64)
        par_pos.append(sorted(int(c) for c in chosen))
    return par_pos


def _hub_dag(rng: np.random.Generator, n: int, n_children: int):
    """A hub at position 0 parenting positions 1..n_children; each child adds
    k ~ U{0,1,2} extra parents among earlier non-hub positions; the remaining
    positions draw k ~ U{0,1,2} parents among all earlier positions."""
    par_pos = [[]]
    for i in range(1, n):
        if i <= n_children:
            cand = np.arange(1, i)
            k = int(rng.integers(0, min(2, cand.size) + 1))
            extra = rng.choice(cand, size=k, replace=False) if k else []
            par_pos.append(sorted([0] + [int(c) for c in extra]))
        else:
            cand = np.arange(0, i)
            k = int(rng.integers(0, min(2, cand.size) + 1))
            extra = rng.choice(cand, size=k, replace=False) if k else []
            par_pos.append(sorted(int(c) for c in extra))
    return par_pos


def _dirichlet_rows(rng: np.random.Generator, rows: int, r: int, alpha: float) -> np.ndarray:
    """rows x r matrix, each row ~ Dirichlet(alpha,...,alpha), every entry > 0."""
    g = rng.gamma(alpha, 1.0, size=(rows, r))
    while True:
        s = g.sum(axis=1, keepdims=True)
        bad = ~np.all(g > 0, axis=1) | ~np.isfinite(s[:, 0]) | (s[:, 0] <= 0)
        if not bad.any():
            break
        g[bad] = rng.gamma(alpha, 1.0, size=(int(bad.sum()), r))
    p = g / g.sum(axis=1, keepdims=True)
    # normalising can still round a tiny share to zero; redraw those rows
    zero = ~np.all(p > 0, axis=1)
    if zero.any():
        p[zero] = _dirichlet_rows(rng, int(zero.sum()), r, alpha)
    return p


# --------------------------------------------------------------------------
# the five workload shapes
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Config:
    key: str
    index: int
    n_nets: int
    n_cases: int
    alpha: float
    cap: int | None           # max clique-table entries accepted (None: no cap)
    cap_low: int | None = None  # lower bound on the largest clique (hub shape)
    description: str = ""


CONFIGS = {
    "C1": Config("C1", 1, 1, 100, 1.0, 4096, None,
                 "24 variables, <=3 parents among all earlier, cards {2,3}, Dirichlet(1); "
                 "100 cases observing 3 variables"),
    "C2": Config("C2", 2, 1, 1000, 0.5, 4_000_000, None,
                 "440 variables, card 3, <=2 parents from the previous 40, Dirichlet(0.5); "
                 "1000 cases observing 5% (22) of the variables"),
    "C3": Config("C3", 3, 1, 500, 0.2, 20_000_000, 5_000_000,
                 "110 variables, hub of 63 states parenting 60 others (+<=2 extra parents), "
                 "cards in {2..63}, Dirichlet(0.2); 500 cases observing 10 variables"),
    "C4": Config("C4", 4, 256, 64, 1.0, 32_768, None,
                 "256 networks of U[50,500] variables, cards {2..6}, <=3 parents from the previous 30, "
                 "Dirichlet(1); 64 cases each observing 4% of the variables"),
    # C4 drawn by rejection alone under the 4e6-entry guard: each network is
    # the first of its seeded draws whose largest clique fits, with every
    # drawn arc kept (no repair)
    "C4G": Config("C4G", 4, 256, 64, 1.0, 4_000_000, None,
                  "256 networks of U[50,500] variables, cards {2..6}, <=3 parents from the previous 30, "
                  "Dirichlet(1), each the first seeded draw whose largest clique is <= 4e6 entries (no arcs "
                  "dropped); 64 cases each observing 4% of the variables"),
    "C5": Config("C5", 5, 8, 4096, 1.0, 4_000_000, None,
                 "8 networks of U[400,1000] variables, cards {2..21}, <=3 parents from the previous 50, "
                 "Dirichlet(1); Poisson arrivals, each query picks a network and observes 2-20%"),
}

_ACCEPTED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "accepted.json")
_accepted_cache = None


def load_accepted() -> dict:
    global _accepted_cache
    if _accepted_cache is None:
        if os.path.exists(_ACCEPTED_PATH):
            with open(_ACCEPTED_PATH) as f:
                _accepted_cache = json.load(f)
        else:
            _accepted_cache = {}
    return _accepted_cache


def _choice_for(key: str, j: int) -> dict:
    return load_accepted().get(key, {}).get(str(j), {"attempt": 0, "card_mode": "uniform", "drop": []})


def make_structure(key: str, j: int = 0, attempt: int = 0, card_mode: str = "uniform", drop=(),
                   return_positions: bool = False):
    """Structure (cards, parents) only; no CPT values.  ``drop`` lists arcs
    (parent_id, child_id) removed after sampling.  With return_positions the
    topological position of every variable id is returned as well."""
    cfg = CONFIGS[key]
    k = cfg.index
    r_dag = _rng(k, j, 0, attempt)
    r_card = _rng(k, j, 1, attempt)
    if key == "C1":
        n = 24
        par_pos = random_dag(r_dag, n, 3, None)
        card_pos = r_card.integers(2, 4, size=n)
    elif key == "C2":
        n = 440
        par_pos = random_dag(r_dag, n, 2, 40)
        card_pos = np.full(n, 3)
    elif key == "C3":
        n = 110
        par_pos = _hub_dag(r_dag, n, 60)
        if card_mode == "uniform":
            card_pos = r_card.integers(2, 64, size=n)
        else:  # P(r) proportional to 1/r on {2..63}
            rs = np.arange(2, 64)
            w = 1.0 / rs
            card_pos = r_card.choice(rs, size=n, p=w / w.sum())
        card_pos[0] = 63
    elif key in ("C4", "C4G"):
        n = int(r_dag.integers(50, 501))
        par_pos = random_dag(r_dag, n, 3, 30)
        card_pos = r_card.integers(2, 7, size=n)
    elif key == "C5":
        n = int(r_dag.integers(400, 1001))
        par_pos = random_dag(r_dag, n, 3, 50)
        card_pos = r_card.integers(2, 22, size=n)
    else:
        raise KeyError(key)
    # variable ids are a seeded permutation of topological positions
    perm = r_dag.permutation(n)          # perm[position] = variable id
    card = np.zeros(n, dtype=np.int32)
    parents = [None] * n
    for pos in range(n):
        v = int(perm[pos])
        card[v] = int(card_pos[pos])
        parents[v] = sorted(int(perm[p]) for p in par_pos[pos])
    dropset = {(int(a), int(b)) for a, b in drop}
    if dropset:
        parents = [[p for p in parents[v] if (p, v) not in dropset] for v in range(n)]
    if return_positions:
        pos_of = np.empty(n, dtype=np.int64)
        pos_of[perm] = np.arange(n)
        return card, parents, pos_of
    return card, parents


def make_net(key: str, j: int = 0, with_cpts: bool = True, choice: dict | None = None) -> Net:
    """Network j of workload ``key`` with the accepted attempt / arc drops."""
    cfg = CONFIGS[key]
    ch = choice if choice is not None else _choice_for(key, j)
    card, parents = make_structure(key, j, ch.get("attempt", 0), ch.get("card_mode", "uniform"),
                                   ch.get("drop", []))
    net = Net(card, parents, [], name=f"{key}.{j}")
    if with_cpts:
        r_cpt = _rng(cfg.index, j, 2, ch.get("attempt", 0))
        for v in range(net.n):
            rows = 1
            for p in parents[v]:
                rows *= int(card[p])
            net.cpt.append(_dirichlet_rows(r_cpt, rows, int(card[v]), cfg.alpha).ravel())
    return net


def _n_observed(key: str, n: int, rng: np.random.Generator | None = None) -> int:
    if key == "C1":
        return 3
    if key == "C2":
        return max(1, int(np.floor(0.05 * n + 0.5)))
    if key == "C3":
        return 10
    if key in ("C4", "C4G"):
        return max(1, int(np.floor(0.04 * n + 0.5)))
    if key == "C5":
        f = float(rng.uniform(0.02, 0.20))
        return max(1, int(np.floor(f * n + 0.5)))
    raise KeyError(key)


def make_cases(key: str, net: Net, j: int = 0, n_cases: int | None = None):
    """Evidence cases: distinct observed variables drawn uniformly without
    replacement, each at a uniformly drawn state.  Every CPT entry is > 0, so
    every such case has P(e) > 0 and no case needs rejecting."""
    cfg = CONFIGS[key]
    rng = _rng(cfg.index, j, 3)
    m = cfg.n_cases if n_cases is None else n_cases
    cases = []
    for _ in range(m):
        k = _n_observed(key, net.n, rng)
        vs = np.sort(rng.choice(net.n, size=k, replace=False)).astype(np.int32)
        st = np.array([int(rng.integers(0, int(net.card[v]))) for v in vs], dtype=np.int32)
        cases.append((vs, st))
    return cases


def forest_offsets(nets) -> np.ndarray:
    """Variable-id offset of each network in a forest built from `nets` in
    order: network k's variables follow those of networks 0..k-1."""
    return np.concatenate([[0], np.cumsum([n.n for n in nets])]).astype(np.int64)


def forest_case(offsets, cases_per_net, s: int):
    """Evidence of one forest slot: case s of every network, ids offset."""
    vs, st = [], []
    for k, cases in enumerate(cases_per_net):
        v, x = cases[s]
        vs.append(np.asarray(v, np.int64) + int(offsets[k]))
        st.append(np.asarray(x, np.int64))
    return (np.concatenate(vs).astype(np.int32) if vs else np.zeros(0, np.int32),
            np.concatenate(st).astype(np.int32) if st else np.zeros(0, np.int32))


def make_arrivals(key: str = "C5", n_queries: int = 4096, n_nets: int = 8):
    """Served-load trace: unit-rate Poisson inter-arrival gaps (scale by 1/lambda
    at replay), each query picking a network uniformly and an observed
    fraction f ~ U[0.02, 0.20]."""
    cfg = CONFIGS[key]
    rng = _rng(cfg.index, 0, 4)
    gaps = rng.exponential(1.0, size=n_queries)
    nets = rng.integers(0, n_nets, size=n_queries)
    fracs = rng.uniform(0.02, 0.20, size=n_queries)
    seeds = rng.integers(0, 2**62, size=n_queries)
    return np.cumsum(gaps), nets.astype(np.int32), fracs, seeds


def case_for_arrival(net: Net, frac: float, seed: int):
    """The evidence case of one arrival of the served trace."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    k = max(1, int(np.floor(frac * net.n + 0.5)))
    vs = np.sort(rng.choice(net.n, size=k, replace=False)).astype(np.int32)
    st = np.array([int(rng.integers(0, int(net.card[v]))) for v in vs], dtype=np.int32)
    return vs, st


def random_small_net(seed: int, n: int, max_card: int = 3, p_max: int = 3, alpha: float = 1.0,
                     window: int | None = None) -> Net:
    """A small random network for property tests (not one of the workloads)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    par_pos = random_dag(rng, n, p_max, window)
    card_pos = rng.integers(2, max_card + 1, size=n)
    perm = rng.permutation(n)
    card = np.zeros(n, dtype=np.int32)
    parents = [None] * n
    for pos in range(n):
        v = int(perm[pos])
        card[v] = int(card_pos[pos])
        parents[v] = sorted(int(perm[p]) for p in par_pos[pos])
    net = Net(card, parents, [])
    for v in range(n):
        rows = 1
        for p in parents[v]:
            rows *= int(card[p])
        net.cpt.append(_dirichlet_rows(rng, rows, int(card[v]), alpha).ravel())
    return net

"""Independent reference computations that pin the oracle.

None of this reuses the oracle's junction-tree arithmetic: it works from the
joint distribution (brute-force enumeration), from the forward-backward
recursion on chains, from the naive-Bayes closed form, and from graph facts
checked with networkx.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import networkx as nx
import numpy as np


def joint(net) -> np.ndarray:
    """Full joint P(x) as an n-dimensional array, axis v = variable v.
    Each CPT is laid out parents in listed order, then the child fastest."""
    n = net.n
    shape = [int(r) for r in net.card]
    P = np.ones(shape, dtype=np.float64)
    for v in range(n):
        fam = list(net.parents[v]) + [v]
        t = np.asarray(net.cpt[v], dtype=np.float64).reshape([shape[u] for u in fam])
        order = np.argsort(fam)
        t = np.transpose(t, order)
        fam_sorted = [fam[i] for i in order]
        bshape = [1] * n
        for u in fam_sorted:
            bshape[u] = shape[u]
        P = P * t.reshape(bshape)
    return P


def brute_force(net, vars_, states):
    """(P(e), posteriors concatenated over variables) by enumeration."""
    P = joint(net)
    idx = [slice(None)] * net.n
    mask = np.ones_like(P)
    for v, s in zip(vars_, states):
        m = np.zeros(int(net.card[v]))
        m[int(s)] = 1.0
        bshape = [1] * net.n
        bshape[int(v)] = int(net.card[v])
        mask = mask * m.reshape(bshape)
    Pe_joint = P * mask
    pe = float(Pe_joint.sum())
    post = []
    for v in range(net.n):
        axes = tuple(a for a in range(net.n) if a != v)
        m = Pe_joint.sum(axis=axes)
        post.append(m / m.sum())
    del idx
    return pe, np.concatenate(post)


def brute_force_joint(net, vars_, states, qvars):
    """P(qvars | e) by enumeration of the joint: the evidence-masked joint
    summed over every other variable, qvars[0] the slowest axis."""
    P = joint(net)
    for v, s in zip(vars_, states):
        m = np.zeros(int(net.card[v]))
        m[int(s)] = 1.0
        bshape = [1] * net.n
        bshape[int(v)] = int(net.card[v])
        P = P * m.reshape(bshape)
    q = [int(x) for x in qvars]
    m = P.sum(axis=tuple(a for a in range(net.n) if a not in q))
    # remaining axes are in ascending variable order; put them in q's order
    m = np.transpose(m, [sorted(q).index(x) for x in q])
    return (m / m.sum()).ravel()


def chain_forward_backward(prior0, trans, obs):
    """Smoothing on a chain X0 -> X1 -> ... -> X_{n-1}.
    prior0[r], trans[t][a, b] = P(X_{t+1}=b | X_t=a), obs = {t: state}.
    Returns (P(e), list of posterior vectors)."""
    n = len(trans) + 1
    def ev(t, r):
        e = np.ones(r)
        if t in obs:
            e = np.zeros(r); e[obs[t]] = 1.0
        return e
    alpha = [None] * n
    alpha[0] = prior0 * ev(0, len(prior0))
    for t in range(1, n):
        alpha[t] = (alpha[t - 1] @ trans[t - 1]) * ev(t, trans[t - 1].shape[1])
    beta = [None] * n
    beta[n - 1] = np.ones(len(alpha[n - 1]))
    for t in range(n - 2, -1, -1):
        beta[t] = trans[t] @ (ev(t + 1, trans[t].shape[1]) * beta[t + 1])
    pe = float(alpha[n - 1].sum())
    return pe, [a * b / pe for a, b in zip(alpha, beta)]


def naive_bayes(prior_h, cond, obs):
    """Hub H with children j, cond[j][h, x] = P(X_j=x | H=h), obs = {j: x}.
    Returns (P(e), P(H|e), {j: P(X_j|e)})."""
    w = prior_h.copy()
    for j, x in obs.items():
        w = w * cond[j][:, x]
    pe = float(w.sum())
    ph = w / pe
    pc = {}
    for j in range(len(cond)):
        if j in obs:
            p = np.zeros(cond[j].shape[1]); p[obs[j]] = 1.0
        else:
            p = ph @ cond[j]
        pc[j] = p
    return pe, ph, pc


def moral_graph(net) -> nx.Graph:
    g = nx.Graph()
    g.add_nodes_from(range(net.n))
    for v in range(net.n):
        ps = list(net.parents[v])
        for p in ps:
            g.add_edge(p, v)
        for a, b in itertools.combinations(ps, 2):
            g.add_edge(a, b)
    return g


def digits(i, card_list):
    """Mixed-radix digits of i, last position fastest."""
    out = [0] * len(card_list)
    for k in range(len(card_list) - 1, -1, -1):
        out[k] = i % card_list[k]
        i //= card_list[k]
    return out


def frac(s: str) -> Fraction:
    return Fraction(s)

"""Helpers shared by the GPU tests: run cases through the HIP library and
through the oracle, and compare."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_2212_04241_amd import fbn

FP64_RTOL = 1e-12     # posteriors and P(e), relative per entry
FP32_ATOL = 1e-5      # posteriors, absolute per entry
FP32_LOGPE_ATOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(net, cases, precision=fbn.FBN_FP64, tile=0, slots=None, jt=None, max_slots=None, layout=0):
    """All cases in one batch.  Returns (post[n, sum card], log_pe[n], status[n], jt)."""
    n = len(cases)
    if jt is None:
        jt = fbn.JT(fbn.net_from_spec(net), precision=precision, max_slots=max_slots or max(n, 1),
                    tile_entries=tile, layout=layout)
    slots = list(range(n)) if slots is None else list(slots)
    fbn.set_evidence_batch(jt, slots, cases)
    lp, st = fbn.calibrate(jt, slots, want_results=True)
    post, lp2, st2 = fbn.query_all(jt, slots, int(np.sum(net.card)))
    assert np.array_equal(st, st2)
    assert np.array_equal(lp[st == 0], lp2[st == 0])
    return post, lp, st, jt


def oracle_run(net, cases, ojt=None):
    ojt = ojt or oracle.compile_net(net)
    out = []
    for v, s in cases:
        lp, post = ojt.query(v, s)
        out.append((lp, post))
    return out, ojt


def check_fp64(post, lp, st, ref, label=""):
    for k, (olp, opost) in enumerate(ref):
        assert st[k] == 0, (label, k, st[k])
        err = np.abs(post[k] - opost)
        bad = err > FP64_RTOL * np.abs(opost) + 1e-300
        assert not bad.any(), (label, k, float(np.max(err / np.maximum(np.abs(opost), 1e-300))))
        assert abs(lp[k] - olp) <= FP64_RTOL * max(1.0, abs(olp)), (label, k, lp[k], olp)


def check_fp32(post, lp, st, ref, label=""):
    worst = 0.0
    for k, (olp, opost) in enumerate(ref):
        assert st[k] == 0, (label, k, st[k])
        e = float(np.max(np.abs(post[k] - opost)))
        worst = max(worst, e)
        assert e <= FP32_ATOL, (label, k, e)
        assert abs(lp[k] - olp) <= FP32_LOGPE_ATOL * max(1.0, abs(olp)), (label, k, lp[k], olp)
    return worst

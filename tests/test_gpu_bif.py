"""GPU parity of a network loaded from BIF text: inference on the library's
BIF reading of the hand-written network against the oracle on the same
network read by the generator's own .fbn parser (the two files are the same
network written by hand in both formats)."""
import os

import numpy as np
import pytest

import fbngen
from paper_2212_04241_amd import fbn
from tests.gpu_util import check_fp32, check_fp64, oracle_run, say

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "bif")


def test_bif_network_matches_oracle():
    with open(os.path.join(GOLD, "commute.fbn")) as f:
        ref_net = fbngen.net_from_text(f.read())
    net = fbn.load_net(os.path.join(GOLD, "commute.bif"))
    # evidence given by names, mapped through the reader's name tables
    named = [[], [("late", "yes")], [("weather", "rain"), ("late", "no")],
             [("slippery", "yes"), ("traffic", "heavy"), ("sprinkler", "on")]]
    cases = []
    for ev in named:
        vs = [fbn.net_find_var(net, v) for v, _ in ev]
        ss = [fbn.net_find_state(net, v, s) for v, (_, s) in zip(vs, ev)]
        cases.append((np.array(vs, np.int32), np.array(ss, np.int32)))
    # and every single-variable observation
    for v in range(ref_net.n):
        for s in range(int(ref_net.card[v])):
            cases.append((np.array([v], np.int32), np.array([s], np.int32)))
    ref, _ = oracle_run(ref_net, cases)
    say("BIF network,", len(cases), "cases")
    cs = int(np.sum(ref_net.card))
    for prec in (fbn.FBN_FP64, fbn.FBN_FP32_RESCALED):
        jt = fbn.JT(net, precision=prec, max_slots=len(cases))
        slots = list(range(len(cases)))
        fbn.set_evidence_batch(jt, slots, cases)
        lp, st = fbn.calibrate(jt, slots, want_results=True)
        post, _, _ = fbn.query_all(jt, slots, cs)
        (check_fp64 if prec == fbn.FBN_FP64 else check_fp32)(post, lp, st, ref, f"bif {prec}")
        jt.free()

"""FP32 trees built with fp64_rerun: a slot whose FP32 messages vanish is
recomputed inside the library on a one-slot FP64 tree of the same network,
and its results are bitwise those of an FP64 tree of the same tile; a slot
whose evidence is impossible reports zero evidence, not underflow; other
slots keep their FP32 results.  Without the option the slot reports
FBN_E_UNDERFLOW."""
import numpy as np
import pytest

import fbngen
import oracle
from paper_2212_04241_amd import fbn
from tests.gpu_util import FP32_ATOL, say

pytestmark = pytest.mark.gpu

# A -> B with P(B = 1 | A) = 1e-60 (below float32's range once scaled), and an
# independent C with P(C = 1) = 0
_NET = ("fbn 1\nvars 3\nvar 0 2 0\nvar 1 2 1 0\nvar 2 2 0\ncpt 0 2\n0.25 0.75\n"
        "cpt 1 4\n1 1e-60 1 1e-60\ncpt 2 2\n1 0\nend\n")
CASES = [([1], [1]),          # FP32 underflow: FP64 gives P(e) = 1e-60
         ([0], [1]),          # ordinary
         ([2], [1]),          # impossible evidence
         ([0, 1], [0, 1])]    # underflow again, two observations


def _fp64_alone(net, case, tile):
    jt = fbn.JT(fbn.net_from_spec(net), precision=fbn.FBN_FP64, max_slots=1, tile_entries=tile)
    fbn.set_evidence(jt, 0, *case)
    lp, st = fbn.calibrate(jt, [0], want_results=True)
    post, _, _ = fbn.query_all(jt, [0], int(np.sum(net.card)))
    jt.free()
    return lp[0], st[0], post[0]


@pytest.mark.parametrize("layout", [fbn.FBN_LAYOUT_PER_SLOT, fbn.FBN_LAYOUT_INTERLEAVED])
def test_underflowed_slots_rerun_in_fp64(layout):
    net = fbngen.net_from_text(_NET)
    cs = int(np.sum(net.card))
    slots = [0, 1, 2, 3]
    say("fp64 rerun, layout", layout)
    plain = fbn.JT(fbn.net_from_spec(net), precision=fbn.FBN_FP32_RESCALED, max_slots=4, layout=layout)
    fbn.set_evidence_batch(plain, slots, CASES)
    _, st = fbn.calibrate(plain, slots, want_results=True)
    assert list(st) == [fbn.FBN_E_UNDERFLOW, 0, fbn.FBN_E_UNDERFLOW, fbn.FBN_E_UNDERFLOW]
    plain.free()
    jt = fbn.JT(fbn.net_from_spec(net), precision=fbn.FBN_FP32_RESCALED, max_slots=4, layout=layout, fp64_rerun=True)
    fbn.set_evidence_batch(jt, slots, CASES)
    lp, st = fbn.calibrate(jt, slots, want_results=True)
    assert list(st) == [0, 0, fbn.FBN_E_ZERO_EVIDENCE, 0]
    post, lp2, st2 = fbn.query_all(jt, slots, cs)
    assert list(st2) == [0, 0, fbn.FBN_E_ZERO_EVIDENCE, 0]
    ojt = oracle.compile_net(net)
    for k in (0, 3):
        flp, fst, fpost = _fp64_alone(net, CASES[k], 0)
        assert fst == 0
        assert lp[k] == flp and lp2[k] == flp and np.array_equal(post[k], fpost), k
        olp, opost = ojt.query(*CASES[k])
        assert abs(lp[k] - olp) <= 1e-12 * abs(olp) and np.all(np.abs(post[k] - opost) <= 1e-12 * np.abs(opost))
    olp, opost = ojt.query(*CASES[1])
    assert np.max(np.abs(post[1] - opost)) <= FP32_ATOL
    # joint read-out of an underflowed slot comes from the FP64 tree
    got = fbn.query_joint(jt, 0, [0, 1], net.card)
    want = oracle.query_joint(ojt, *CASES[0], [0, 1])
    assert np.all(np.abs(got - want) <= 1e-12 * np.abs(want) + 1e-300)
    # the single-variable query call reruns too
    m = fbn.query_marginals(jt, 3, [0], net.card)
    assert np.array_equal(m, post[3][:2])
    jt.free()

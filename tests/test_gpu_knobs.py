"""The per-slot layout's two tuning knobs on the device.  Slots per layer
workgroup only changes which slots share a workgroup's index arithmetic:
every slot's sums keep their order, so results are bitwise equal for every
cap (1, 2, 4, 8) and for the library's own choice.  The finaliser block size
changes how a large separator's posterior sums are split, so results move
by rounding only: FP64 within the oracle's relative bar, FP32 within its
absolute bar, on C2 (whose large separators are finalised in blocks) and C5
networks."""
import numpy as np
import pytest

import fbngen
from paper_2212_04241_amd import fbn
from tests.gpu_util import check_fp32, check_fp64, oracle_run, say

pytestmark = pytest.mark.gpu
PS = fbn.FBN_LAYOUT_PER_SLOT


def _run(net, cases, precision, tile=0, **knobs):
    n = len(cases)
    jt = fbn.JT(fbn.net_from_spec(net), precision=precision, max_slots=n, layout=PS, tile_entries=tile, **knobs)
    slots = list(range(n))
    fbn.set_evidence_batch(jt, slots, cases)
    lp, st = fbn.calibrate(jt, slots, want_results=True)
    post, _, _ = fbn.query_all(jt, slots, int(np.sum(net.card)))
    jt.free()
    return post, lp, st


@pytest.mark.parametrize("precision", [fbn.FBN_FP64, fbn.FBN_FP32_RESCALED])
@pytest.mark.parametrize("cfg,tile", [("C2", 0), ("C2", 512), ("C5", 2048)])
def test_slots_per_block_is_bitwise_invariant(precision, cfg, tile):
    net = fbngen.make_net(cfg, 0)
    cases = fbngen.make_cases(cfg, net)[:11] if cfg != "C5" else \
        [fbngen.case_for_arrival(net, 0.02 + 0.018 * k, 700 + k) for k in range(11)]
    say(cfg, "slots_per_block", precision, tile)
    ref = _run(net, cases, precision, tile)
    for cap in (1, 2, 4, 8):
        got = _run(net, cases, precision, tile, slots_per_block=cap)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (cfg, cap)


@pytest.mark.parametrize("precision", [fbn.FBN_FP64, fbn.FBN_FP32_RESCALED])
def test_finaliser_block_size_keeps_oracle_parity_c2(precision):
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:6]
    ref, _ = oracle_run(net, cases)
    say("C2 fin_block", precision)
    base = _run(net, cases, precision)
    for fb in (64, 1000, 2048):
        post, lp, st = _run(net, cases, precision, fin_block=fb)
        if precision == fbn.FBN_FP64:
            check_fp64(post, lp, st, ref, f"fin_block {fb}")
        else:
            check_fp32(post, lp, st, ref, f"fin_block {fb}")
        # P(e) does not depend on the posterior sums' split
        assert np.array_equal(lp, base[1]), fb


def test_tuned_knobs_keep_oracle_parity_c5():
    net = fbngen.make_net("C5", 1)
    cases = [fbngen.case_for_arrival(net, 0.05 + 0.01 * k, 900 + k) for k in range(8)]
    ref, _ = oracle_run(net, cases)
    say("C5 knobs")
    for kb in ({"slots_per_block": 2, "fin_block": 1024}, {"slots_per_block": 8, "fin_block": 64}):
        post, lp, st = _run(net, cases, fbn.FBN_FP32_RESCALED, 2048, **kb)
        check_fp32(post, lp, st, ref, str(kb))

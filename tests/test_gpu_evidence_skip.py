"""The shrinking reduction of the per-slot layout: a table entry that a
slot's evidence zeroes is neither read nor written for that slot (its
working-table entry is never stored), so a calibration streams only the
evidence-consistent entries.  Results must be bitwise those of streaming
every entry (the zeroed entries add exact zeros in the same order), for
every batch width the kernels take (1, 2, 4, 8 slots per workgroup) and for
packed and split tiles, and stale working-table entries left by an earlier
case must never be read.  Against the oracle: the usual bars on C2, C3 and
C5 networks in both precisions."""
import numpy as np
import pytest

import fbngen
from paper_2212_04241_amd import fbn
from tests.gpu_util import check_fp32, check_fp64, oracle_run, say

pytestmark = pytest.mark.gpu
PS = fbn.FBN_LAYOUT_PER_SLOT


def _run(net, cases, precision, dense, tile=0, slots=None, jt=None):
    n = len(cases)
    if jt is None:
        jt = fbn.JT(fbn.net_from_spec(net), precision=precision, max_slots=max(n, 8), layout=PS, tile_entries=tile,
                    shrink_evidence=not dense)
    slots = list(range(n)) if slots is None else slots
    fbn.set_evidence_batch(jt, slots, cases)
    lp, st = fbn.calibrate(jt, slots, want_results=True)
    post, _, _ = fbn.query_all(jt, slots, int(np.sum(net.card)))
    return post, lp, st, jt


@pytest.mark.parametrize("precision", [fbn.FBN_FP64, fbn.FBN_FP32_RESCALED])
@pytest.mark.parametrize("tile", [0, 100, 2048])
def test_skip_equals_dense_bitwise_c2(precision, tile):
    net = fbngen.make_net("C2", 0)
    cases = fbngen.make_cases("C2", net)[:9]
    say("C2 skip vs dense", precision, tile)
    for n in (1, 2, 5, 9):               # one, two, four and eight slots per workgroup
        a = _run(net, cases[:n], precision, False, tile)
        b = _run(net, cases[:n], precision, True, tile)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), n
        a[3].free()
        b[3].free()


def test_skip_equals_dense_bitwise_c5_and_oracle():
    net = fbngen.make_net("C5", 7)
    rng = np.random.default_rng(3)
    cases = [fbngen.case_for_arrival(net, f, int(rng.integers(0, 2**62))) for f in (0.02, 0.08, 0.14, 0.2)]
    ref, _ = oracle_run(net, cases)
    say("C5 net 7 skip vs dense")
    for prec in (fbn.FBN_FP64, fbn.FBN_FP32_RESCALED):
        a = _run(net, cases, prec, False, 2048)
        b = _run(net, cases, prec, True, 2048)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), prec
        (check_fp64 if prec == fbn.FBN_FP64 else check_fp32)(a[0], a[1], a[2], ref, f"C5 skip {prec}")


@pytest.mark.timeout(600)
def test_skip_c3_against_oracle():
    net = fbngen.make_net("C3", 0)
    cases = fbngen.make_cases("C3", net)[:2]
    ref, _ = oracle_run(net, cases)
    say("C3 skip")
    a = _run(net, cases, fbn.FBN_FP64, False)
    check_fp64(a[0], a[1], a[2], ref, "C3 fp64 skip")
    a[3].free()
    b = _run(net, cases, fbn.FBN_FP32_RESCALED, False)
    check_fp32(b[0], b[1], b[2], ref, "C3 fp32 skip")
    c = _run(net, cases, fbn.FBN_FP32_RESCALED, True)
    assert np.array_equal(b[0], c[0]) and np.array_equal(b[1], c[1])


def test_stale_working_tables_are_never_read():
    """A slot first calibrated with evidence that keeps entries live, then with
    evidence that zeroes them: the second result equals a fresh slot's."""
    net = fbngen.make_net("C2", 0)
    rng = np.random.default_rng(9)
    cases = fbngen.make_cases("C2", net)[:4]
    # heavier evidence: a third of the variables observed
    heavy = []
    for _ in range(4):
        vs = np.sort(rng.choice(net.n, size=net.n // 3, replace=False)).astype(np.int32)
        heavy.append((vs, np.array([int(rng.integers(0, int(net.card[v]))) for v in vs], np.int32)))
    empty = [(np.zeros(0, np.int32), np.zeros(0, np.int32))] * 4
    for prec in (fbn.FBN_FP64, fbn.FBN_FP32_RESCALED):
        jt = fbn.JT(fbn.net_from_spec(net), precision=prec, max_slots=4, layout=PS, shrink_evidence=True)
        _run(net, empty, prec, False, jt=jt)            # every psi entry written
        got = _run(net, heavy, prec, False, jt=jt)       # most entries now skipped
        _run(net, cases, prec, False, jt=jt)
        again = _run(net, heavy, prec, False, jt=jt)
        fresh = _run(net, heavy, prec, False)
        for r in (got, again):
            assert np.array_equal(r[0], fresh[0]) and np.array_equal(r[1], fresh[1]), prec
        ref, _ = oracle_run(net, heavy)
        (check_fp64 if prec == fbn.FBN_FP64 else check_fp32)(got[0], got[1], got[2], ref, f"heavy {prec}")
        jt.free()

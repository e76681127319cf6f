"""The GPU parity bar itself (tests/parity.py), exercised on the CPU with the
oracle on both sides: identical events pass; an entry moved to a neighbouring
bin, an event binned in the wrong place on one side only, or a weight
changed fail.  (The mistakes are planted in a copy of the oracle's output.)"""
import copy

import numpy as np
import pytest

from tests import parity


def _as_gpu(o, n):
    """The oracle's output in the layout of the GPU binding's results."""
    rn = o["rec"]["n"]
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum(rn)
    return dict(sum_i=o["sum_i"].T.copy(), sum_d=o["sum_d"].T.copy(), hash=o["hash"].copy(), hist=o["hist"].copy(),
                rec_offsets=off,
                rec_p=np.concatenate([o["rec"]["p"][e, :rn[e]] for e in range(n)]),
                rec_pid=np.concatenate([o["rec"]["pid"][e, :rn[e]] for e in range(n)]).astype(np.int8),
                rec_col=np.concatenate([o["rec"]["col"][e, :rn[e]] for e in range(n)]).astype(np.uint16),
                rec_acol=np.concatenate([o["rec"]["acol"][e, :rn[e]] for e in range(n)]).astype(np.uint16))


@pytest.fixture(scope="module")
def run(oracle):
    n = 600
    o = oracle.generate(5, 0, n, 91.2, 1.0, 64, records=True)
    return o, _as_gpu(o, n), n


def test_identical_events_pass(run):
    o, g, n = run
    rep, same = parity.compare(g, o, 91.2, n)
    parity.assert_parity(rep)
    assert same.all() and rep["entry_excess"] <= 0 and rep["entry_self_excess"] <= 0


@pytest.mark.parametrize("h", [0, 2, 7])
def test_an_entry_moved_to_the_next_bin_fails(run, h):
    o, g, n = run
    g = copy.deepcopy(g)
    cell = g["hist"][h]
    b = int(np.flatnonzero(cell[1:-2, 2] > 0)[0]) + 1  # a filled bin with a neighbour
    cell[b, 2] -= 1
    cell[b + 1, 2] += 1
    rep, _ = parity.compare(g, o, 91.2, n)
    with pytest.raises(AssertionError):
        parity.assert_parity(rep)


def test_misbinned_on_one_side_fails_even_if_chi2_is_small(run):
    # the GPU histogram fills one event's tau into the underflow bin instead
    o, g, n = run
    g = copy.deepcopy(g)
    e = int(np.flatnonzero((o["sum_i"][:, 1] == 1) & (o["sum_d"][:, 4] > 0.05))[0])
    b = int(parity.bin_index(np.array([o["sum_d"][e, 4]]), 2)[0])
    w = o["sum_d"][e, 0]
    for src, dst in ((b, 0),):
        g["hist"][2, src] -= [w, w * w, 1]
        g["hist"][2, dst] += [w, w * w, 1]
    rep, _ = parity.compare(g, o, 91.2, n)
    assert rep["chi2_ndf"] < 1.5  # the weighted chi^2 alone would not notice
    with pytest.raises(AssertionError):
        parity.assert_parity(rep)


def test_a_differing_event_may_move_its_own_entries(run):
    # an event that is not identical on both sides (different hash) may sit
    # in different bins: its entries are allowed to move
    o, g, n = run
    g = copy.deepcopy(g)
    e = int(np.flatnonzero((o["sum_i"][:, 1] == 1) & (o["sum_d"][:, 4] > 0.05))[0])
    g["hash"][e] ^= 1
    b = int(parity.bin_index(np.array([o["sum_d"][e, 4]]), 2)[0])
    w = o["sum_d"][e, 0]
    g["sum_d"][4, e] = 0.0  # the GPU's tau of this event is 0: underflow... bin 1
    nb = int(parity.bin_index(np.array([0.0]), 2)[0])
    g["hist"][2, b] -= [w, w * w, 1]
    g["hist"][2, nb] += [w, w * w, 1]
    rep, same = parity.compare(g, o, 91.2, n)
    assert not same[e]
    assert rep["entry_excess"] <= 0 and rep["entry_self_excess"] <= 0


def test_isr_rows_are_checked(oracle):
    n = 800
    o = oracle.isr_generate(4, 0, n, 1960.0, 91.2, 1.0, 64, records=True)
    g = _as_gpu(o, n)
    rep, same = parity.compare(g, o, 91.2, n, isr=True)
    parity.assert_parity(rep)
    g2 = copy.deepcopy(g)
    cell = g2["hist"][0]
    b = int(np.flatnonzero(cell[1:-2, 2] > 0)[0]) + 1
    cell[b, 2] -= 1
    cell[b + 1, 2] += 1
    rep, _ = parity.compare(g2, o, 91.2, n, isr=True)
    with pytest.raises(AssertionError):
        parity.assert_parity(rep)

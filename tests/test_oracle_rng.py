"""Pins of the oracle's random numbers: Philox4x32-10 known answers, the exact
u(0,1) conversion, and the keyed-draw contract."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(oracle):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, expect in rows:
        assert list(oracle.philox(ctr, key)) == expect


def test_uniform_is_exact_and_open(oracle):
    assert oracle.uniform(0, 0) == 2.0 ** -53
    assert oracle.uniform(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    # the low 12 bits of the high word are discarded; the rest is a 52-bit integer
    assert oracle.uniform(0xFFF, 0) == 2.0 ** -53
    assert oracle.uniform(1 << 12, 0) == (2.0 * 2.0 ** 32 + 1.0) * 2.0 ** -53
    assert oracle.uniform(0, 1) == 3.0 * 2.0 ** -53


def test_draw_counter_layout(oracle):
    seed = (7 << 32) | 5
    event = (3 << 32) | 11
    out = oracle.draw(seed, event, 9, oracle.P_TRIAL, 0x12345)
    ref = oracle.philox([11, 3, 9, (oracle.P_TRIAL << 24) | 0x12345], [5, 7])
    assert list(out) == list(ref)


def test_uniform_statistics(oracle):
    L = oracle.lib()
    n = 200_000
    us = np.empty(n)
    for i in range(n // 2):
        w = oracle.draw(1, i, 0, oracle.P_ACCEPT, 0)
        us[2 * i] = oracle.uniform(w[0], w[1])
        us[2 * i + 1] = oracle.uniform(w[2], w[3])
    assert us.min() > 0.0 and us.max() < 1.0
    assert abs(us.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(us.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
    counts, _ = np.histogram(us, bins=50, range=(0, 1))
    exp = n / 50
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 49 + 5 * np.sqrt(2 * 49)
    assert L is not None

"""Pins of the oracle's counter RNG (Philox4x32-10, reading R5) and of the
mating draw (R6), against published test vectors and distribution checks."""
import os

import numpy as np
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle_core):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle_core.philox(np.array([ctr], dtype=np.uint32), np.array(key, dtype=np.uint32))
        assert [int(x) for x in got[0]] == want


def test_philox_counter_sensitivity(oracle_core):
    # every counter word and key word changes the output block
    base = np.zeros((1, 4), dtype=np.uint32)
    key = np.zeros(2, dtype=np.uint32)
    ref = oracle_core.philox(base, key)[0]
    for w in range(4):
        c = base.copy()
        c[0, w] = 1
        assert not np.array_equal(oracle_core.philox(c, key)[0], ref)
    for w in range(2):
        k = key.copy()
        k[w] = 1
        assert not np.array_equal(oracle_core.philox(base, k)[0], ref)


def test_philox_uniformity(oracle_core):
    n = 200_000
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint32)
    ctr[:, 3] = (3 << 24) | (1 << 16)
    out = oracle_core.philox(ctr, np.array([7, 0], dtype=np.uint32))
    words = out.reshape(-1)
    u = (words >> 8).astype(np.float64) / 16777216.0
    hist, _ = np.histogram(u, bins=64, range=(0.0, 1.0))
    chi2 = stats.chisquare(hist)
    assert chi2.pvalue > 1e-4
    # every bit is balanced
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(0)
    assert np.all(np.abs(bits - 0.5) < 0.01)


def test_mate_distinct_in_range_and_uniform(oracle_core):
    rng = np.random.default_rng(1)
    t = 7
    counts = np.zeros((t, t), dtype=np.int64)
    for _ in range(30000):
        w0, w1 = (int(x) for x in rng.integers(0, 2**32, size=2))
        r1, r2 = oracle_core.mate(w0, w1, t)
        assert 0 <= r1 < t and 0 <= r2 < t and r1 != r2
        counts[r1, r2] += 1
    off = counts[~np.eye(t, dtype=bool)]
    assert stats.chisquare(off).pvalue > 1e-4


def test_mate_extremes(oracle_core):
    # w = 0 picks position 0; w = 2^32 - 1 picks the last position (hi32(w t))
    assert oracle_core.mate(0, 0, 10) == (0, 1)
    assert oracle_core.mate(0xFFFFFFFF, 0xFFFFFFFF, 10) == (9, 8)
    assert oracle_core.mate(0xFFFFFFFF, 0, 10) == (9, 0)
    # a single-member neighbourhood mates the member with itself
    assert oracle_core.mate(123456, 654321, 1) == (0, 0)

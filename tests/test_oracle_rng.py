"""Pins of the oracle's random streams.

Philox4x32-10 is pinned to the published known-answer vectors of Salmon et
al., "Parallel random numbers: as easy as 1, 2, 3" (SC'11), as distributed
with the authors' Random123 library (kat_vectors, philox4x32 with 10 rounds).
The uniform conversions and the slot layout are pinned bit-exactly from the
raw Philox words, and statistically (KS test, moments, independence).
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle

def _load_kat():
    """counter (4 words), key (2 words) -> output (4 words), from the golden file."""
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = []
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        ctr, key, out = ([int(w, 16) for w in part.split()] for part in line.split("|"))
        rows.append((ctr, key, out))
    return rows


KAT = _load_kat()


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    assert oracle.philox4x32_10(ctr, key) == expect


def test_slot_layout_and_conversion_bit_exact():
    """Slot s reads Philox block s//2, words 2(s%2) (high) and 2(s%2)+1 (low);
    the counter is (block, packet, wavelength, model) and the key is the seed
    split into (low, high) 32-bit halves."""
    seed = 0x0123456789ABCDEF
    for packet, lam, model in [(0, 0, 0), (7, 3, 1), (123456, 63, 255)]:
        for slot in range(12):
            w = oracle.philox4x32_10([slot // 2, packet, lam, model],
                                     [seed & 0xFFFFFFFF, seed >> 32])
            hi, lo = w[2 * (slot % 2)], w[2 * (slot % 2) + 1]
            word = (hi << 32) | lo
            # exact: ((word >> 12) + 1/2) * 2^-52 is representable in FP64
            u64 = ((word >> 12) * 2 + 1) / float(1 << 53)
            assert oracle.uniform64(seed, packet, lam, model, slot) == u64
            u32 = ((hi >> 9) * 2 + 1) / float(1 << 24)
            assert oracle.uniform32(seed, packet, lam, model, slot) == np.float32(u32)
            assert 0.0 < u64 < 1.0 and 0.0 < u32 < 1.0


def test_uniforms_statistics():
    n = 20000
    u = np.array([oracle.uniform64(0, i, 0, 0, 0) for i in range(n)])
    v = np.array([oracle.uniform64(0, i, 0, 0, 1) for i in range(n)])
    w = np.array([oracle.uniform64(0, i, 1, 0, 0) for i in range(n)])
    for x in (u, v, w):
        assert stats.kstest(x, "uniform").pvalue > 1e-4
        assert abs(x.mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)
    # different slots / wavelengths are uncorrelated
    for a, b in ((u, v), (u, w)):
        assert abs(np.corrcoef(a, b)[0, 1]) < 4 / np.sqrt(n)
    # different seeds give different streams
    assert oracle.uniform64(1, 0, 0, 0, 0) != oracle.uniform64(0, 0, 0, 0, 0)
    assert oracle.uniform64(1 << 32, 0, 0, 0, 0) != oracle.uniform64(0, 0, 0, 0, 0)

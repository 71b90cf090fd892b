"""Pins for the oracle's Philox4x64-10 and its draw from alias tables."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden",
                      "philox4x64_10_kat.txt")
M64 = (1 << 64) - 1


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat_rows())
def test_philox_known_answers(ctr, key, want):
    # published Random123 vectors (tests/golden), independent of any code here
    got = oracle.philox4x64_10(ctr, key)
    assert [int(x) for x in got] == want


def test_philox_matches_numpy_bitgenerator():
    # numpy's Philox bit generator is Philox4x64-10; it increments its
    # counter before producing a block, so counter c-1 yields block c.
    g = np.random.default_rng(123)
    for _ in range(200):
        ctr = [int(x) for x in g.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr[0] |= 1  # keep c-1 free of borrow for a simple construction
        key = [int(x) for x in g.integers(0, 2**63, size=2, dtype=np.int64)]
        bg = np.random.Philox(counter=[ctr[0] - 1] + ctr[1:], key=key)
        want = [int(x) for x in bg.random_raw(4)]
        assert [int(x) for x in oracle.philox4x64_10(ctr, key)] == want


def test_philox_sample_counter_layout():
    # the sampler's block for sample l of query qid is counter (l, qid, 0, 0)
    # and key (seed, 0); consecutive l differ (no reuse of streams)
    seed = 0xABCDEF
    blocks = {tuple(int(v) for v in oracle.philox4x64_10([l, 3, 0, 0],
                                                          [seed, 0]))
              for l in range(1000)}
    assert len(blocks) == 1000


def test_draw_uses_top_bits_for_slot_and_low_bits_for_coin():
    # a 4-slot table: slot u = top 2 bits; u is kept when coin < thr[u]
    thr = np.array([5, 0, 7, 0], np.uint32)
    al = np.array([1, 1, 1, 3], np.uint32)
    for u in range(4):
        for coin in (0, 4, 5, 6, 7, (1 << 31) - 1):
            U = (u << 62) | (0x5A5A << 31) | coin  # bits 31..61 ignored
            want = u if coin < thr[u] else int(al[u])
            assert oracle.draw(thr, al, U) == want
    # one slot: every word returns slot 0 or its alias
    assert oracle.draw(np.array([0], np.uint32), np.array([0], np.uint32),
                       M64) == 0

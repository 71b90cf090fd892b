"""GPU checks of the score accumulation (the pair form of the score update of Alg. 3)
through mad_debug_accumulate, against a numpy group-by of the same pairs:
every key's sum of rne(v 2^F) in int64, bit for bit.  Cases reach the
paths that sampled inputs rarely do: one key taking half of the pairs,
thousands of distinct keys in one hash bin (the reduction's LDS table
overflows and the bin is split), no closed pair at all, one pair, negative
and vanishing increments, and sizes with a second partition level."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EMPTY = -1  # ~0 as int64
M64 = (1 << 64) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mad_gpu(gpu):
    import paper_1506_03872_amd as mad
    mad.lib()
    return mad


def expected(keys, vals, F):
    keep = keys != EMPTY
    k = keys[keep]
    inc = np.rint(np.ldexp(vals[keep].astype(np.float64), F)).astype(np.int64)
    uk, inv = np.unique(k, return_inverse=True)
    x = np.zeros(len(uk), dtype=np.int64)
    np.add.at(x, inv, inc)
    return uk, x


def run(mad, keys, vals, F):
    import torch
    tk = torch.from_numpy(np.ascontiguousarray(keys, dtype=np.int64)).cuda()
    tv = torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float32)).cuda()
    gk, gx = mad.debug_accumulate(tk, tv, F)
    ek, ex = expected(keys, vals, F)
    assert np.array_equal(gk, ek)
    assert np.array_equal(gx, ex)
    # the inputs are left as they were
    assert np.array_equal(tk.cpu().numpy(), keys)
    return len(gk)


def mix64(z):
    """The 64-bit finaliser the partition hashes keys with (Stafford's
    variant 13, as in SplitMix64), to build keys that share a bin."""
    z = np.asarray(z, dtype=np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def test_random_keys_with_open_samples(mad_gpu):
    g = np.random.default_rng(1)
    n = 300_000
    keys = g.integers(0, 100_000, n).astype(np.int64)
    keys[g.random(n) < 0.2] = EMPTY
    vals = g.standard_normal(n).astype(np.float32)
    say("distinct", run(mad_gpu, keys, vals, 20))


def test_one_hot_key(mad_gpu):
    g = np.random.default_rng(2)
    n = 200_000
    keys = g.integers(0, 10**9, n).astype(np.int64)
    keys[g.random(n) < 0.5] = 123456789
    vals = g.standard_normal(n).astype(np.float32)
    run(mad_gpu, keys, vals, 24)


def test_many_distinct_keys_in_one_bin(mad_gpu):
    # n = 4096 pairs make 8 first-level bins (the top 3 hash bits) and no
    # second level: 3000 distinct keys whose hash starts with 000 all land
    # in bin 0, far beyond one reduction table
    g = np.random.default_rng(3)
    cand = g.integers(0, 1 << 40, 40_000, dtype=np.int64)
    h = mix64(cand.astype(np.uint64))
    same = np.unique(cand[(h >> np.uint64(61)) == 0])[:3000]
    assert len(same) == 3000
    n = 4096
    keys = np.concatenate([same, g.choice(same, n - len(same))])
    g.shuffle(keys)
    vals = g.standard_normal(n).astype(np.float32)
    assert run(mad_gpu, keys, vals, 18) == 3000


def test_second_partition_level(mad_gpu):
    g = np.random.default_rng(4)
    n = 2_000_000  # 12 hash bits: 256 bins, each split 16 ways
    keys = g.integers(0, 5_000_000, n).astype(np.int64)
    keys[g.random(n) < 0.3] = EMPTY
    vals = (g.standard_normal(n) * 1e-3).astype(np.float32)
    run(mad_gpu, keys, vals, 30)


def test_edge_cases(mad_gpu):
    g = np.random.default_rng(5)
    run(mad_gpu, np.array([7], np.int64), np.array([1.5], np.float32), 3)
    assert run(mad_gpu, np.full(1000, EMPTY, np.int64),
               np.ones(1000, np.float32), 5) == 0
    assert run(mad_gpu, np.zeros(0, np.int64), np.zeros(0, np.float32), 5) == 0
    # vanishing and cancelling increments: keys stay, with x = 0
    keys = np.array([5, 5, 9, 11, 11], np.int64)
    vals = np.array([1.0, -1.0, 1e-30, 2.0, -0.5], np.float32)
    assert run(mad_gpu, keys, vals, 10) == 3
    keys = g.integers(0, 50, 5000).astype(np.int64)
    vals = g.standard_normal(5000).astype(np.float32)
    run(mad_gpu, keys, vals, 40)


@pytest.mark.parametrize("slots", [1024, 4096, 8192])
def test_reduce_table_sizes(mad_gpu, slots):
    # the reduction's LDS table is sized to the bins (1024 slots; 4096 or
    # 8192 for bins of many pairs, at s near 1e9): each size forced on
    # random keys and on 10000 distinct keys of one bin, more than any of
    # the tables holds below its probe limit, so every size splits the bin
    g = np.random.default_rng(6)
    os.environ["MAD_ACC_SLOTS"] = str(slots)
    try:
        say("slots", slots)
        keys = g.integers(0, 400_000, 600_000).astype(np.int64)
        keys[g.random(len(keys)) < 0.1] = EMPTY
        vals = g.standard_normal(len(keys)).astype(np.float32)
        run(mad_gpu, keys, vals, 22)
        # n = 16384 pairs: 32 first-level bins (top 5 hash bits)
        cand = np.unique(g.integers(0, 1 << 40, 600_000, dtype=np.int64))
        h = mix64(cand.astype(np.uint64))
        same = cand[(h >> np.uint64(59)) == 0][:10_000]
        assert len(same) == 10_000
        n = 16384
        keys = np.concatenate([same, g.choice(same, n - len(same))])
        g.shuffle(keys)
        vals = g.standard_normal(n).astype(np.float32)
        assert run(mad_gpu, keys, vals, 18) == 10_000
    finally:
        del os.environ["MAD_ACC_SLOTS"]


def test_two_splits_after_the_first_partition(mad_gpu):
    # 3.6e7 pairs: 2^17 final bins of ~275 pairs, 9 bits below the first
    # level's 8, taken in two splits (5 + 4 bits)
    g = np.random.default_rng(7)
    n = 36_000_000
    keys = g.integers(0, 40_000_000_000, n, dtype=np.int64)
    keys[: n // 4] = g.integers(0, 3_000_000, n // 4)   # repeated keys
    keys[g.random(n) < 0.15] = EMPTY
    vals = (g.standard_normal(n) * 1e-2).astype(np.float32)
    say("distinct", run(mad_gpu, keys, vals, 28))

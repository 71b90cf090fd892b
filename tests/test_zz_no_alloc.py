"""GPU check of the allocation-free score accumulation (mad_accumulate_noalloc)
through the C ABI: on two calls in a row, the second with fewer pairs, its
output must equal mad_debug_accumulate's on the same pairs, key for key and
sum for sum (exact int64), with nothing left over from the first call."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EMPTY = -1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mad_gpu(gpu):
    import paper_1506_03872_amd as mad
    mad.lib()
    return mad


def _pairs(n, nkeys, seed):
    g = np.random.default_rng(seed)
    keys = g.integers(0, nkeys, n).astype(np.int64)
    keys[g.random(n) < 0.15] = EMPTY
    vals = g.standard_normal(n).astype(np.float32)
    return keys, vals


def _noalloc(mad, keys, vals, F):
    import torch
    n = len(keys)
    tk = torch.from_numpy(keys).cuda()
    tv = torch.from_numpy(vals).cuda()
    ok = torch.full((max(n, 1),), -7, dtype=torch.int64, device="cuda")
    ox = torch.full((max(n, 1),), -7, dtype=torch.int64, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = mad.lib().mad_accumulate_noalloc(
        C.c_void_p(tk.data_ptr()), C.c_void_p(tv.data_ptr()), n, F,
        C.c_void_p(ok.data_ptr()), C.c_void_p(ox.data_ptr()),
        C.c_void_p(cnt.data_ptr()), stream)
    assert rc == mad.MAD_OK, mad.lib().mad_last_error()
    torch.cuda.synchronize()
    m = int(cnt.item())
    k = ok[:m].cpu().numpy()
    x = ox[:m].cpu().numpy()
    o = np.argsort(k, kind="stable")
    assert np.array_equal(tk.cpu().numpy(), keys)  # inputs unchanged
    return k[o], x[o]


def _reference(mad, keys, vals, F):
    import torch
    tk = torch.from_numpy(keys).cuda()
    tv = torch.from_numpy(vals).cuda()
    return mad.debug_accumulate(tk, tv, F)


def test_noalloc_matches_allocating_entry_point(mad_gpu):
    mad = mad_gpu
    for n, nkeys, seed, F in ((262_144, 40_000, 1, 22), (5_000, 3_000, 2, 30)):
        say("noalloc n=%d keys<%d" % (n, nkeys))
        keys, vals = _pairs(n, nkeys, seed)
        gk, gx = _noalloc(mad, keys, vals, F)
        rk, rx = _reference(mad, keys, vals, F)
        assert np.array_equal(gk, rk) and np.array_equal(gx, rx)


def test_noalloc_edges(mad_gpu):
    import torch
    mad = mad_gpu
    # no pairs: zero keys
    keys = np.zeros(0, np.int64)
    vals = np.zeros(0, np.float32)
    gk, _ = _noalloc(mad, keys, vals, 20)
    assert len(gk) == 0
    # every pair open
    keys = np.full(100, EMPTY, np.int64)
    vals = np.ones(100, np.float32)
    gk, _ = _noalloc(mad, keys, vals, 20)
    assert len(gk) == 0
    # above the limit: rejected before any work
    big = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc = mad.lib().mad_accumulate_noalloc(
        C.c_void_p(big.data_ptr()), C.c_void_p(big.data_ptr()),
        (1 << 18) + 1, 20, C.c_void_p(big.data_ptr()),
        C.c_void_p(big.data_ptr()), C.c_void_p(big.data_ptr()), None)
    assert rc == mad.MAD_EINVAL
    assert b"static workspace" in mad.lib().mad_last_error()

"""GPU checks of the exact sparse brute force (exhaustive t-MAD of sparse
inputs, the exact baseline of Sec. 5.3) against the oracle's sparse FP64
product: the same top t by |c| (swaps allowed only among pairs whose |c|
lie within the fp32 error scale of the t-th value), c within 1e-5 relative,
with every split of the coordinates into a dense heavy part and listed
light wedges, and every precision of the heavy part's filter."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mad_gpu(gpu):
    import paper_1506_03872_amd as mad
    mad.lib()
    return mad


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _c64(a, b, keys, n):
    """Exact c of the pairs by sparse merges in FP64."""
    out = np.empty(len(keys))
    for q, kk in enumerate(keys.tolist()):
        i, j = divmod(kk, n)
        ia = a[1][a[0][i]:a[0][i + 1]]
        va = a[2][a[0][i]:a[0][i + 1]]
        ib = b[1][b[0][j]:b[0][j + 1]]
        vb = b[2][b[0][j]:b[0][j + 1]]
        _, xa, xb = np.intersect1d(ia, ib, return_indices=True)
        out[q] = float(np.dot(va[xa].astype(np.float64),
                              vb[xb].astype(np.float64)))
    return out


def _scale(a, b, keys, n):
    out = np.empty(len(keys))
    for q, kk in enumerate(keys.tolist()):
        i, j = divmod(kk, n)
        ia = a[1][a[0][i]:a[0][i + 1]]
        va = a[2][a[0][i]:a[0][i + 1]]
        ib = b[1][b[0][j]:b[0][j + 1]]
        vb = b[2][b[0][j]:b[0][j + 1]]
        _, xa, xb = np.intersect1d(ia, ib, return_indices=True)
        out[q] = float(np.abs(va[xa].astype(np.float64) *
                              vb[xb].astype(np.float64)).sum())
    return out


def _check(mad, a, b, m, n, d, t, prec=0, heavy=0):
    res, st = mad.bruteforce_topk_csr(tuple(to_dev(x) for x in a),
                                      tuple(to_dev(x) for x in b), m, n, d,
                                      t, precision=prec, heavy=heavy)
    say("stats", {k: (round(v, 3) if isinstance(v, float) else v)
                  for k, v in st.items()})
    k_ex, c_ex = oracle.exact_topk_sparse(a, b, m, n, d, t)
    got = res["i"].cpu().numpy() * n + res["j"].cpu().numpy()
    assert len(got) == len(k_ex)
    c64 = _c64(a, b, got, n)
    gc = res["c"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gc - c64) <= TOL * np.abs(c64))
    if not np.array_equal(got, k_ex):
        tau = np.abs(c_ex).min()
        sc = _scale(a, b, got, n)
        ex = set(k_ex.tolist())
        for kk, c, s in zip(got.tolist(), c64.tolist(), sc.tolist()):
            if kk not in ex:
                assert abs(abs(c) - tau) <= 2 * TOL * s, kk
    return st


@pytest.mark.parametrize("heavy", [0, 64, 512])
def test_powerlaw_reduced_c3(mad_gpu, heavy):
    # the C3 distributions (Zipf(1.5) coordinates over d = 1e5, lognormal
    # values with random signs) at 0.5% of the vector counts
    cfg, data = workloads.make("C3", seed=0, scale=0.005)
    a, b, m, n = data["a"], data["b"], data["m"], data["n"]
    st = _check(mad_gpu, a, b, m, n, cfg["d"], 200, prec=1, heavy=heavy)
    assert st["heavy"] >= 1
    if heavy:
        assert st["heavy"] == heavy


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_precisions_of_the_heavy_filter(mad_gpu, prec):
    cfg, data = workloads.make("C3", seed=1, scale=0.003)
    a, b, m, n = data["a"], data["b"], data["m"], data["n"]
    _check(mad_gpu, a, b, m, n, cfg["d"], 100, prec=prec, heavy=128)


@pytest.mark.parametrize("heavy", [0, 1, 7, 29])
def test_ragged_inputs(mad_gpu, heavy):
    # empty vectors, unused coordinates, stored zeros; every split from all
    # light to all heavy
    a, b, m, n, d = workloads.ragged_csr(300, 400, 30, seed=14, density=0.2)
    _check(mad_gpu, a, b, m, n, d, 60, prec=0, heavy=heavy)


def test_arguments(mad_gpu):
    mad = mad_gpu
    a, b, m, n, d = workloads.ragged_csr(50, 40, 10, seed=15)
    ga = tuple(to_dev(x) for x in a)
    gb = tuple(to_dev(x) for x in b)
    with pytest.raises(mad.MadError):
        mad.bruteforce_topk_csr(ga, gb, m, n, d, 0)
    with pytest.raises(mad.MadError):
        mad.bruteforce_topk_csr(ga, gb, m, n, d, 5, precision=9)
    bad_idx = a[1].copy()
    bad_idx[3] = d + 5                       # coordinate out of range
    gbad = (ga[0], to_dev(bad_idx), ga[2])
    with pytest.raises(mad.MadError) as ei:
        mad.bruteforce_topk_csr(gbad, gb, m, n, d, 5)
    assert ei.value.code == mad.MAD_EINVAL
    # no shared coordinate: nothing to return
    z = (np.arange(m + 1, dtype=np.int64), np.zeros(m, np.int32),
         np.ones(m, np.float32))
    w = (np.arange(n + 1, dtype=np.int64), np.ones(n, np.int32),
         np.ones(n, np.float32))
    res, _ = mad.bruteforce_topk_csr(tuple(to_dev(x) for x in z),
                                     tuple(to_dev(x) for x in w), m, n, 2, 5)
    assert len(res["i"]) == 0

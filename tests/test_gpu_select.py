"""GPU parity of Alg. 2's selections (the t' largest scores, then the t
largest |c|, ties by key) when the coarse bin that holds the boundary
element is long.

The library refines such a boundary list with one full-grid radix pass (on
the primary values when they differ inside the bin, on the keys when they
are all equal) before the single-workgroup exact selection.  Each case here
is chosen so that the boundary bin has more than 4096 elements, which the
test checks on the oracle's results; the candidate set must match the
oracle's bit for bit, and so must the final pairs where c is exact."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5
REFINE_MIN = 4096


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


def fbin(p):
    """The coarse digit of a positive score: its highest set bit and the 5
    bits below it (1/32-octave bins)."""
    p = int(p)
    msb = p.bit_length() - 1
    mant = (p >> (msb - 5)) if msb >= 5 else (p << (5 - msb))
    return msb * 32 + (mant & 31)


def boundary(ox, tp):
    """(length of the bin that holds the tp-th largest positive score,
    number of distinct scores in it)"""
    pos = np.sort(ox[ox > 0])[::-1]
    b = fbin(pos[tp - 1])
    inbin = pos[[fbin(v) == b for v in pos]]
    return len(inbin), len(np.unique(inbin))


def _unit_csr():
    m, n, d = 3000, 2500, 2000
    a = workloads.powerlaw_csr(m, d, 20, 1.5, seed=11, role=0)
    b = workloads.powerlaw_csr(n, d, 20, 1.5, seed=11, role=1)
    return (a[0], a[1], np.ones_like(a[2])), (b[0], b[1], np.ones_like(b[2])), m, n, d


# (kind, inputs, s, t', t, whether the boundary scores are all equal)
CASES = {
    # x values differ inside the bin: the refinement digit is one of x's
    "dense_x_digit": ("dense",
                      lambda: workloads.dense_gaussian(3001, 2049, 37, seed=3)[:2],
                      1_000_000, 100_000, 10, False),
    # one x value in the bin: the refinement digit is one of the keys
    "dense_key_digit": ("dense",
                        lambda: workloads.binary(700, 900, 48, density=0.3, seed=5),
                        100_000, 5000, 20, True),
    "csr_key_digit_small_rem": ("csr", _unit_csr, 200_000, 1000, 10, True),
    "csr_key_digit_large_rem": ("csr", _unit_csr, 200_000, 20_000, 10, True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_long_boundary_candidates_bitexact(mad_gpu, name):
    kind, gen, s, tp, t, tied = CASES[name]
    if kind == "dense":
        A, B = (np.ascontiguousarray(x, np.float32) for x in gen())
        m, n = A.shape[0], B.shape[0]
        op = oracle.Plan.dense(A, B)
        gp = mad_gpu.Plan.dense(to_dev(A), to_dev(B))
    else:
        a, b, m, n, d = gen()
        op = oracle.Plan.csr(a[0], a[1], a[2], m, b[0], b[1], b[2], n, d)
        gp = mad_gpu.Plan.csr(tuple(to_dev(x) for x in a),
                              tuple(to_dev(x) for x in b), m, n, d)
        A = workloads.csr_to_dense(a[0], a[1], a[2], m, d)
        B = workloads.csr_to_dense(b[0], b[1], b[2], n, d)
    o = op.topk(seed=42, s=s, t_prime=tp, t=t)
    ok, ox, _ = op.scores(seed=42, s=s, F=o["F"])
    nbin, ndistinct = boundary(ox, tp)
    say("case", name, "s", s, "t'", tp, "boundary bin", nbin, "distinct", ndistinct)
    assert nbin > REFINE_MIN          # the case does reach the refinement
    assert (ndistinct == 1) == tied
    g = gp.topk(t=t, s=s, t_prime=tp, seed=42)
    assert gp.stats()["n_pos"] == o["n_pos"]
    ck, cx, cc = gp.candidates()
    order = np.argsort(o["tp_key"])
    assert len(ck) == tp
    assert np.array_equal(ck, o["tp_key"][order])
    assert np.array_equal(cx, o["tp_x"][order])
    err = np.abs(cc.astype(np.float64) - o["tp_c"][order])
    scale = (np.abs(A[ck // n].astype(np.float64)) *
             np.abs(B[ck % n].astype(np.float64))).sum(1)
    assert np.all(err <= TOL * scale + 1e-30)
    # the final top t: every key's c within tolerance, and the set equal to
    # the oracle's up to swaps at the t-th |c|
    gkey = g["i"].cpu().numpy() * n + g["j"].cpu().numpy()
    assert len(gkey) == len(o["key"])
    c64 = (A[gkey // n].astype(np.float64) * B[gkey % n].astype(np.float64)).sum(1)
    if not np.array_equal(gkey, o["key"]):
        tau = np.abs(o["c"]).min()
        inset = set(o["key"].tolist())
        for kk, c in zip(gkey.tolist(), c64.tolist()):
            if kk not in inset:
                sc = (np.abs(A[kk // n].astype(np.float64)) *
                      np.abs(B[kk % n].astype(np.float64))).sum()
                assert abs(abs(c) - tau) <= 2 * TOL * sc, kk
    gp.close()


def test_long_boundary_repeat_calls_agree(mad_gpu):
    """The refined list and its counters start from zero on each call: a
    long-boundary call after a short-boundary one, and again, gives the same
    candidates."""
    A, B = (np.ascontiguousarray(x, np.float32)
            for x in workloads.binary(700, 900, 48, density=0.3, seed=5))
    gp = mad_gpu.Plan.dense(to_dev(A), to_dev(B))
    runs = []
    for tp in (5000, 100, 5000, 5000):
        gp.topk(t=20, s=100_000, t_prime=tp, seed=42)
        runs.append(gp.candidates()[0])
    assert np.array_equal(runs[0], runs[2]) and np.array_equal(runs[0], runs[3])
    assert len(runs[1]) == 100
    gp.close()


def test_long_final_boundary_exact(mad_gpu):
    """The final selection (top t by |c|, ties by key) with 12,124 candidates
    tied at the t-th |c|: 0/1 inputs make every c an integer, exact in fp32
    as in FP64, so the t pairs and their order must equal the oracle's."""
    A, B = (np.ascontiguousarray(x, np.float32)
            for x in workloads.binary(700, 900, 48, density=0.3, seed=5))
    n = B.shape[0]
    s, tp, t = 1_000_000, 100_000, 20_000
    op = oracle.Plan.dense(A, B)
    o = op.topk(seed=42, s=s, t_prime=tp, t=t)
    c = np.abs(o["tp_c"])
    tv = np.sort(c)[::-1][t - 1]
    say("final boundary: t-th |c|", tv, "tied", int((c == tv).sum()))
    assert (c == tv).sum() > REFINE_MIN
    gp = mad_gpu.Plan.dense(to_dev(A), to_dev(B))
    for rep in range(2):  # the second call starts from the first's state
        g = gp.topk(t=t, s=s, t_prime=tp, seed=42)
        gkey = g["i"].cpu().numpy() * n + g["j"].cpu().numpy()
        assert np.array_equal(gkey, o["key"]), rep
        assert np.array_equal(g["c"].cpu().numpy().astype(np.float64), o["c"]), rep
    gp.close()

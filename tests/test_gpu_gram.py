"""GPU parity of the Gram variant (Sec. 3.2.2, B = A): symmetrised scores
x_ij + x_ji on i < j with the diagonal left out, against the oracle's Gram
mode, for dense and sparse inputs.  Scores and candidates bit-exact; the
final pairs as for the general plan."""
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


def _compare(gp, op, Ad, m, s, tp, t, seed=17):
    g = gp.topk(t=t, s=s, t_prime=tp, seed=seed)
    o = op.topk(seed=seed, s=s, t_prime=tp, t=t)
    gk, gx, F = gp.scores()
    ok, ox, closed = op.scores(seed=seed, s=s, F=o["F"])
    assert F == o["F"]
    assert np.array_equal(gk, ok) and np.array_equal(gx, ox)
    assert np.all(gk // m < gk % m)
    st = gp.stats()
    assert st["closed"] == closed and st["n_pos"] == o["n_pos"]
    ck, cx, _ = gp.candidates()
    order = np.argsort(o["tp_key"])
    assert np.array_equal(ck, o["tp_key"][order])
    assert np.array_equal(cx, o["tp_x"][order])
    gi = g["i"].cpu().numpy()
    gj = g["j"].cpu().numpy()
    assert np.all(gi < gj)
    key = gi * m + gj
    assert len(key) == len(o["key"])
    c64 = (Ad[gi].astype(np.float64) * Ad[gj].astype(np.float64)).sum(1)
    sc = (np.abs(Ad[gi].astype(np.float64)) *
          np.abs(Ad[gj].astype(np.float64))).sum(1)
    gc = g["c"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gc - c64) <= TOL * sc + 1e-30)
    if np.array_equal(key, o["key"]):
        # x reports (x_ij + x_ji) / 2
        ox = np.ldexp(o["x"].astype(np.float64), -o["F"] - 1).astype(np.float32)
        assert np.array_equal(g["x"].cpu().numpy(), ox)
    else:
        tau = np.abs(o["c"]).min()
        okeys = set(o["key"].tolist())
        for kk, c, scv in zip(key.tolist(), c64.tolist(), sc.tolist()):
            if kk not in okeys:
                assert abs(abs(c) - tau) <= 2 * TOL * scv


def test_gram_dense_matches_oracle(mad_gpu):
    A, _ = workloads.dense_gaussian(900, 1, 30, seed=41)
    m = A.shape[0]
    Ad = to_dev(A)
    gp = mad_gpu.Plan.dense(Ad, Ad, flags=mad_gpu.MAD_FLAG_GRAM)
    op = oracle.Plan.dense(A, A.copy())
    op.set_gram(True)
    for s, tp, t in ((300_000, 500, 20), (20_000, 10**6, 10)):
        say("gram dense", s, tp, t)
        _compare(gp, op, A, m, s, tp, t)
    gp.close()


def test_gram_sparse_matches_oracle(mad_gpu):
    A, _ = workloads.binary(1500, 1, 300, density=0.04, seed=42)
    a = workloads.dense_to_csr(A)
    m, d = A.shape
    ta = tuple(to_dev(x) for x in a)
    gp = mad_gpu.Plan.csr(ta, ta, m, m, d, flags=mad_gpu.MAD_FLAG_GRAM)
    op = oracle.Plan.csr(a[0], a[1], a[2], m, a[0], a[1], a[2], m, d)
    op.set_gram(True)
    say("gram sparse")
    _compare(gp, op, A, m, 200_000, 2000, 50)
    gp.close()


def test_gram_needs_equal_inputs(mad_gpu):
    A, B = workloads.dense_gaussian(100, 100, 8, seed=43)
    with pytest.raises(mad_gpu.MadError):
        mad_gpu.Plan.dense(to_dev(A), to_dev(B), flags=mad_gpu.MAD_FLAG_GRAM)

"""GPU parity of the squared variant (Sec. 3.2.3: B = A symmetric, C = A^2):
every closed sample updates x_ij and x_kk', the scores are symmetrised with
the diagonal left out.  Against the oracle's squared mode, dense and sparse:
scores X and candidates bit-exact, the final pairs as for the general plan,
x reported as the symmetrised entry."""
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


def _compare(gp, op, A, s, tp, t, seed=23):
    m = A.shape[0]
    g = gp.topk(t=t, s=s, t_prime=tp, seed=seed)
    o = op.topk(seed=seed, s=s, t_prime=tp, t=t)
    assert gp.fix_exponent(s) == o["F"] == op.fix_exponent(s)
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
    A64 = A.astype(np.float64)
    c64 = (A64[gi] * A64[gj]).sum(1)        # (A^2)_ij for symmetric A
    gc = g["c"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gc - c64) <= TOL * np.abs(c64) + 1e-30)
    if np.array_equal(key, o["key"]):
        # the stored score is four times the symmetrised entry
        ox2 = np.ldexp(o["x"].astype(np.float64), -o["F"] - 2).astype(np.float32)
        assert np.array_equal(g["x"].cpu().numpy(), ox2)
    else:
        sc = (np.abs(A64[gi]) * np.abs(A64[gj])).sum(1)
        tau = np.abs(o["c"]).min()
        okeys = set(o["key"].tolist())
        for kk, c, scv in zip(key.tolist(), c64.tolist(), sc.tolist()):
            if kk not in okeys:
                assert abs(abs(c) - tau) <= 2 * TOL * scv


def _oracle_square(A, csr=None):
    m = A.shape[0]
    if csr is None:
        op = oracle.Plan.dense(A, A.copy())
    else:
        op = oracle.Plan.csr(*csr, m, *csr, m, m)
    op.set_square(True)
    return op


@pytest.mark.parametrize("order", [0, 1])
def test_square_dense_matches_oracle(mad_gpu, order):
    mad = mad_gpu
    A = workloads.symmetric(700, density=0.3, seed=51)
    Ad = to_dev(A)
    gp = mad.Plan.dense(Ad, Ad, flags=mad.MAD_FLAG_SQUARE)
    gp.set_option(mad.MAD_OPT_SAMPLER_ORDER, order)
    op = _oracle_square(A)
    for s, tp, t in ((300_000, 500, 20), (20_000, 10**6, 10)):
        say("square dense", order, s, tp, t)
        _compare(gp, op, A, s, tp, t)
    gp.close()


def test_square_dense_pipeline_option_runs_in_k_order(mad_gpu):
    # order 2 (one pair per sample) falls back to the k order here
    mad = mad_gpu
    A = workloads.symmetric(500, density=0.2, seed=52)
    Ad = to_dev(A)
    gp = mad.Plan.dense(Ad, Ad, flags=mad.MAD_FLAG_SQUARE)
    gp.set_option(mad.MAD_OPT_SAMPLER_ORDER, 2)
    _compare(gp, _oracle_square(A), A, 100_000, 400, 15)
    gp.close()


def test_square_sparse_matches_oracle(mad_gpu):
    mad = mad_gpu
    A = workloads.symmetric(2000, density=0.01, seed=53, weighted=True)
    csr = workloads.dense_to_csr(A)
    ta = tuple(to_dev(x) for x in csr)
    m = A.shape[0]
    gp = mad.Plan.csr(ta, ta, m, m, m, flags=mad.MAD_FLAG_SQUARE)
    say("square sparse nnz", len(csr[1]))
    _compare(gp, _oracle_square(A, csr), A, 400_000, 3000, 40)
    gp.close()


def test_square_argument_checks(mad_gpu):
    mad = mad_gpu
    A = workloads.symmetric(64, density=0.3, seed=54)
    N = A.copy()
    N[3, 5] += 1.0                       # not symmetric
    with pytest.raises(mad.MadError) as ei:
        Nd = to_dev(N)
        mad.Plan.dense(Nd, Nd, flags=mad.MAD_FLAG_SQUARE)
    assert ei.value.code == mad.MAD_EINVAL
    with pytest.raises(mad.MadError):    # B must be the same array
        mad.Plan.dense(to_dev(A), to_dev(A), flags=mad.MAD_FLAG_SQUARE)
    R = np.ascontiguousarray(A[:, :32])  # m != d
    with pytest.raises(mad.MadError):
        Rd = to_dev(R)
        mad.Plan.dense(Rd, Rd, flags=mad.MAD_FLAG_SQUARE)
    csr = workloads.dense_to_csr(N)
    tn = tuple(to_dev(x) for x in csr)
    with pytest.raises(mad.MadError) as ei:
        mad.Plan.csr(tn, tn, 64, 64, 64, flags=mad.MAD_FLAG_SQUARE)
    assert ei.value.code == mad.MAD_EINVAL
    Ad = to_dev(A)
    gp = mad.Plan.dense(Ad, Ad, flags=mad.MAD_FLAG_SQUARE)
    with pytest.raises(mad.MadError) as ei:
        gp.set_option(mad.MAD_OPT_ACCUM, mad.MAD_ACCUM_HASH)
    assert ei.value.code == mad.MAD_EUNSUPPORTED
    gp.close()

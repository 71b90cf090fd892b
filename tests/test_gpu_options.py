"""GPU parity of every launch choice of a MAD plan against the oracle.

The score matrix X can be built from per-sample pairs or by hash atomics,
and dense samples can run in index order, grouped by k, or in the three
passes grouped by k, by i and by j, in chunks of any power-of-two size.  None of these may change a result, so under each the
score table X and the candidate set Omega_t' must equal the oracle's bit for
bit, and the returned top t must agree with it (c within 1e-5 relative).
The chunked case uses chunks far smaller than the default so that one call
spans many ordering chunks and ends in a partial one, as a run of more than
2^28 samples does at the default chunk."""
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


def _check_run(gp, op, A, B, s, tp, t, seed):
    g = gp.topk(t=t, s=s, t_prime=tp, seed=seed)
    o = op.topk(seed=seed, s=s, t_prime=tp, t=t)
    gk, gx, F = gp.scores()
    ok, ox, _ = op.scores(seed=seed, s=s, F=o["F"])
    assert F == o["F"]
    assert np.array_equal(gk, ok) and np.array_equal(gx, ox)
    st = gp.stats()
    assert st["closed"] == o["closed"] and st["n_pos"] == o["n_pos"]
    ck, cx, _ = gp.candidates()
    order = np.argsort(o["tp_key"])
    assert np.array_equal(ck, o["tp_key"][order])
    assert np.array_equal(cx, o["tp_x"][order])
    n = B.shape[0]
    gkey = g["i"].cpu().numpy() * n + g["j"].cpu().numpy()
    assert np.array_equal(gkey, o["key"])
    c = g["c"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(c - o["c"]) <= TOL * np.abs(o["c"]))


DENSE = {
    "ragged": lambda: workloads.dense_gaussian(3001, 2049, 37, seed=3),
    "zeros": lambda: _with_zeros(),
}


def _with_zeros():
    A, B = workloads.tiny(1200, 1100, 20, seed=7)
    A[A < -1.0] = 0.0
    B[B > 1.2] = 0.0
    A[5] = 0.0
    B[:, 3] = 0.0
    return A, B


# (accumulation, sampler order, ordering chunk); order 2 with the hash form
# runs as order 1
SETTINGS = [(0, 2, 1 << 28), (0, 2, 1 << 12), (1, 2, 1 << 28),
            (1, 1, 1 << 28), (0, 0, 1 << 28), (1, 0, 1 << 28),
            (0, 1, 1 << 12), (1, 1, 1 << 13), (0, 1, 1 << 28)]


@pytest.mark.parametrize("name", list(DENSE))
@pytest.mark.parametrize("setting", SETTINGS)
def test_dense_launch_choices_bitexact(mad_gpu, name, setting):
    mad = mad_gpu
    A, B = DENSE[name]()
    acc, order, chunk = setting
    gp = mad.Plan.dense(to_dev(A), to_dev(B))
    gp.set_option(mad.MAD_OPT_ACCUM, acc)
    gp.set_option(mad.MAD_OPT_SAMPLER_ORDER, order)
    gp.set_option(mad.MAD_OPT_ORDER_CHUNK, chunk)
    assert gp.get_option(mad.MAD_OPT_ACCUM) == acc
    assert gp.get_option(mad.MAD_OPT_SAMPLER_ORDER) == order
    assert gp.get_option(mad.MAD_OPT_ORDER_CHUNK) == chunk
    op = oracle.Plan.dense(A, B)
    for s, tp, t in ((100_003, 300, 10), (9_000, 10**6, 4)):
        say(name, setting, "s", s)
        _check_run(gp, op, A, B, s, tp, t, seed=17)
    gp.close()


def test_many_ordering_chunks_bitexact(mad_gpu):
    # 2.5e6 samples in chunks of 2^20: two full chunks and a partial one
    mad = mad_gpu
    A, B = workloads.dense_gaussian(4000, 3500, 24, seed=21)
    gp = mad.Plan.dense(to_dev(A), to_dev(B))
    gp.set_option(mad.MAD_OPT_ORDER_CHUNK, 1 << 20)
    op = oracle.Plan.dense(A, B)
    say("s 2.5e6 chunk 2^20")
    _check_run(gp, op, A, B, 2_500_000, 2000, 20, seed=3)
    gp.close()


def test_switching_choices_on_one_plan(mad_gpu):
    # the same plan, re-run under every setting in turn, keeps its result
    mad = mad_gpu
    A, B = workloads.dense_gaussian(900, 800, 16, seed=22)
    gp = mad.Plan.dense(to_dev(A), to_dev(B))
    op = oracle.Plan.dense(A, B)
    for acc, order, chunk in SETTINGS + [(0, 2, 1 << 28)]:
        gp.set_option(mad.MAD_OPT_ACCUM, acc)
        gp.set_option(mad.MAD_OPT_SAMPLER_ORDER, order)
        gp.set_option(mad.MAD_OPT_ORDER_CHUNK, chunk)
        _check_run(gp, op, A, B, 40_000, 500, 8, seed=acc + 2 * order)
    gp.close()


@pytest.mark.parametrize("acc", [0, 1])
def test_sparse_accumulation_forms_bitexact(mad_gpu, acc):
    mad = mad_gpu
    a, b, m, n, d = workloads.ragged_csr(700, 900, 60, seed=9, density=0.15)
    ga = tuple(to_dev(x) for x in a)
    gb = tuple(to_dev(x) for x in b)
    gp = mad.Plan.csr(ga, gb, m, n, d)
    gp.set_option(mad.MAD_OPT_ACCUM, acc)
    op = oracle.Plan.csr(*a, m, *b, n, d)
    A = workloads.csr_to_dense(*a, m, d)
    B = workloads.csr_to_dense(*b, n, d)
    _check_run(gp, op, A, B, 200_000, 1000, 12, seed=4)
    with pytest.raises(mad.MadError) as ei:
        gp.set_option(mad.MAD_OPT_SAMPLER_ORDER, 0)
    assert ei.value.code == mad.MAD_EUNSUPPORTED
    gp.close()


def test_option_validation(mad_gpu):
    mad = mad_gpu
    A, B = workloads.dense_gaussian(200, 300, 16, seed=9)
    gp = mad.Plan.dense(to_dev(A), to_dev(B))
    for opt, bad in ((mad.MAD_OPT_ACCUM, 2), (mad.MAD_OPT_SAMPLER_ORDER, 5),
                     (mad.MAD_OPT_ORDER_CHUNK, 3000),
                     (mad.MAD_OPT_ORDER_CHUNK, 1 << 11),
                     (mad.MAD_OPT_ORDER_CHUNK, 1 << 29), (77, 0)):
        with pytest.raises(mad.MadError) as ei:
            gp.set_option(opt, bad)
        assert ei.value.code == mad.MAD_EINVAL
    gp.close()
    mp = mad.MipsPlan.create(to_dev(A))
    with pytest.raises(mad.MadError):
        mp.set_option(mad.MAD_OPT_ACCUM, 0)
    mp.close()

"""GPU checks of repeated table builds of one dense plan: after each
refresh (the inputs changed in place, other GPU work run in between) the
plan's norms, tables, sample stream and results equal those of a fresh plan
on the same inputs."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


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


def _same_plan_state(mad, gp, A, B, m, n, d):
    fp = mad.Plan.dense(to_dev(A), to_dev(B))
    for x, y in zip(gp.norms(), fp.norms()):
        assert np.array_equal(x, y)
    for which, idx in ((0, 0), (1, 0), (1, d - 1), (2, 3), (3, 0), (3, m - 1)):
        for x, y in zip(gp.table(which, idx), fp.table(which, idx)):
            assert np.array_equal(x, y), (which, idx)
    F = fp.fix_exponent(200_000)
    assert gp.fix_exponent(200_000) == F
    g1 = gp.samples(seed=2, l0=0, count=10_000, F=F)
    g2 = fp.samples(seed=2, l0=0, count=10_000, F=F)
    for key in ("k", "i", "j", "kp", "inc"):
        assert np.array_equal(g1[key], g2[key]), key
    r1 = gp.topk(t=20, s=200_000, t_prime=800, seed=6)
    r2 = fp.topk(t=20, s=200_000, t_prime=800, seed=6)
    for k in ("i", "j", "c", "x"):
        assert np.array_equal(r1[k].cpu().numpy(), r2[k].cpu().numpy()), k
    fp.close()


@pytest.mark.parametrize("flags", ["checked", "unchecked"])
def test_refreshes_match_fresh_plans(mad_gpu, flags):
    import torch
    m, n, d = 3000, 2600, 100  # column tables of 4096 slots, d <= 512 rows
    A, B = workloads.dense_gaussian(m, n, d, seed=31)
    tA, tB = to_dev(A), to_dev(B)
    fl = mad_gpu.MAD_FLAG_NO_CHECK if flags == "unchecked" else 0
    gp = mad_gpu.Plan.dense(tA, tB, flags=fl)
    g = np.random.default_rng(32)
    for rep in range(3):
        say("refresh", rep, flags)
        A = g.standard_normal((m, d)).astype(np.float32)
        B = (g.standard_normal((n, d)) * (rep + 1)).astype(np.float32)
        A[rep] = 0.0  # an empty vector
        tA.copy_(torch.from_numpy(A))
        tB.copy_(torch.from_numpy(B))
        torch.cuda.synchronize()
        gp.refresh()
        gp.topk(t=5, s=10_000, t_prime=50, seed=rep)  # eager work between
        torch.cuda.synchronize()
        _same_plan_state(mad_gpu, gp, A, B, m, n, d)
    gp.close()

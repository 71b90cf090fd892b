"""GPU checks of the low-precision verification pattern: bf16 / fp8-e4m3
candidate filtering with an a-priori error bound, then fp32 verification of
the survivors.  The filter is certified, so the final top t must equal the
fp32-verification result bit for bit (indices, c and x), while fewer
candidates reach the fp32 pass; and every result is also checked against
the oracle's (same pairs, c within 1e-5 relative of its FP64 value)."""
import sys

import numpy as np
import pytest

import oracle
import workloads

TOL = 1e-5

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


def _run(mad, A, B, prec, t, s, tp, seed=5):
    p = mad.Plan.dense(to_dev(A), to_dev(B))
    if prec:
        p.set_verify_precision(prec)
    r = p.topk(t=t, s=s, t_prime=tp, seed=seed)
    vs = p.verify_stats()
    st = p.stats()
    p.close()
    return ({k: v.cpu().numpy() for k, v in r.items()}, vs, st)


CASES = {
    "planted_wide": lambda: workloads.planted(3000, 20000, 256, 200, seed=2,
                                              sigma_mult=(8.0, 10.0),
                                              workload="planted_wide")[:2],
    "ragged_d": lambda: workloads.planted(2500, 6000, 100, 100, seed=3)[:2],
    "integers": lambda: tuple(
        np.random.default_rng(4).integers(-6, 7, size=sh).astype(np.float32)
        for sh in ((1500, 72), (1700, 72))),
}


@pytest.mark.parametrize("name", list(CASES))
def test_lowp_filter_keeps_fp32_result(mad_gpu, name):
    A, B = CASES[name]()
    t, s, tp = 50, 2_000_000, 4000
    ref, vs32, st32 = _run(mad_gpu, A, B, 0, t, s, tp)
    assert vs32["n_reranked"] == vs32["n_cand"] == st32["n_cand"]
    o = None
    for prec in (mad_gpu.MAD_BF16, mad_gpu.MAD_FP8_E4M3):
        got, vs, st = _run(mad_gpu, A, B, prec, t, s, tp)
        say(name, "prec", prec, "cand", vs["n_cand"], "fp32 re-ranked",
            vs["n_reranked"])
        assert vs["n_cand"] == vs32["n_cand"]
        assert st["n_cand"] == vs32["n_cand"]
        assert vs["n_reranked"] <= vs["n_cand"]
        for k in ("i", "j", "c", "x"):
            assert np.array_equal(got[k], ref[k]), (prec, k)
        if prec == mad_gpu.MAD_BF16 and name != "integers":
            assert vs["n_reranked"] < vs["n_cand"] // 2
        if o is None:
            o = oracle.Plan.dense(A, B).topk(seed=5, s=s, t_prime=tp, t=t)
        _check_oracle(A, B, got, o)


def _check_oracle(A, B, got, o):
    """The low-precision run against the oracle's run (same seed, s, t'
    and t): the same candidates feed the same exact top t, whose c agree
    within 1e-5 of the FP64 value."""
    n = B.shape[0]
    gkey = got["i"].astype(np.int64) * n + got["j"]
    assert len(gkey) == len(o["key"])
    c64 = (A[gkey // n].astype(np.float64) *
           B[gkey % n].astype(np.float64)).sum(1)
    assert np.all(np.abs(got["c"].astype(np.float64) - c64)
                  <= TOL * np.abs(c64))
    if np.array_equal(gkey, o["key"]):
        assert np.array_equal(got["x"].astype(np.float64),
                              np.ldexp(o["x"].astype(np.float64), -o["F"])
                              .astype(np.float32).astype(np.float64))
        return
    # otherwise only swaps at the t-th |c| within the fp32 error scale
    tau = np.abs(o["c"]).min()
    scale = (np.abs(A[gkey // n].astype(np.float64)) *
             np.abs(B[gkey % n].astype(np.float64))).sum(1)
    for kk, c, sc in zip(gkey.tolist(), c64.tolist(), scale.tolist()):
        if kk not in set(o["key"].tolist()):
            assert abs(abs(c) - tau) <= 2 * TOL * sc, kk


def test_precision_setting_validation(mad_gpu):
    A, B = workloads.dense_gaussian(200, 300, 16, seed=9)
    p = mad_gpu.Plan.dense(to_dev(A), to_dev(B))
    with pytest.raises(mad_gpu.MadError):
        p.set_verify_precision(7)
    p.set_verify_precision(mad_gpu.MAD_BF16)
    p.refresh()  # rebuilds the copies
    r = p.topk(t=5, s=20000, t_prime=100)
    p.set_verify_precision(mad_gpu.MAD_FP32)
    r2 = p.topk(t=5, s=20000, t_prime=100)
    assert np.array_equal(r["i"].cpu().numpy(), r2["i"].cpu().numpy())
    p.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_screen_error_within_its_bound(mad_gpu, prec):
    # every candidate's bf16 / fp8 value c^ lies within its a-priori margin
    # of the fp32 product, measured here against FP64 (the fp32 rounding is
    # far below the margin's own slack)
    import torch
    A, B = CASES["planted_wide"]()
    p = mad_gpu.Plan.dense(to_dev(A), to_dev(B))
    p.set_verify_precision(prec)
    p.topk(t=50, s=2_000_000, t_prime=4000, seed=5)
    xk, xx, _ = p.scores()           # Omega_t': the top t' of X
    pos = xx > 0
    keys = xk[pos][np.lexsort((xk[pos], -xx[pos]))][:4000]
    ch, mg = p.lowp_screen(torch.from_numpy(keys).cuda())
    n = B.shape[0]
    c64 = (A[keys // n].astype(np.float64) *
           B[keys % n].astype(np.float64)).sum(1)
    err = np.abs(ch.astype(np.float64) - c64)
    say("prec", prec, "pairs", len(keys), "max err/bound",
        float((err / mg).max()))
    assert len(keys) > 1000
    assert np.all(err <= mg)
    p.close()

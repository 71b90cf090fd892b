"""GPU parity of sparse (CSR) plans against the CPU oracle, through the C ABI.

Bar as for dense plans: norms and alias tables (thresholds, and the item ids
of each slot and of its alias) bit-exact, per-sample streams and the score
table X bit-exact, the candidate set Omega_t' bit-exact, c within 1e-5 of
sum_k |a_ik b_jk|, the final top t equal up to swaps within that tolerance
at the t-th value.  Cases cover tables of more than 512 items (one
workgroup per table on the GPU), empty vectors and coordinates, explicit
zeros, d = 1, and a dense input given as CSR (which must reproduce the
dense plan's samples)."""
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


def _powerlaw():
    m, n, d = 3000, 2500, 2000
    a = workloads.powerlaw_csr(m, d, 20, 1.5, seed=11, role=0)
    b = workloads.powerlaw_csr(n, d, 20, 1.5, seed=11, role=1)
    return a, b, m, n, d


def _ragged():
    g = np.random.default_rng(12)
    m, n, d = 800, 700, 1500
    A = g.standard_normal((m, d)).astype(np.float32)
    B = g.standard_normal((n, d)).astype(np.float32)
    dens_a = g.uniform(0.0, 0.05, size=m)
    dens_b = g.uniform(0.0, 0.05, size=n)
    A[g.random((m, d)) > dens_a[:, None]] = 0.0
    B[g.random((n, d)) > dens_b[:, None]] = 0.0
    A[3] = 0.0                                     # empty vector
    A[7, :900] = g.standard_normal(900)            # a vector of > 512 entries
    B[:, 5] = 0.0                                  # an empty coordinate
    B[11, 100:700] = g.standard_normal(600)
    return (workloads.dense_to_csr(A), workloads.dense_to_csr(B), m, n, d)


def _explicit_zeros():
    a, b, m, n, d = _powerlaw()
    av = a[2].copy()
    av[::7] = 0.0                                  # stored zeros: weight 0
    bv = b[2].copy()
    bv[::5] = -0.0
    return (a[0], a[1], av), (b[0], b[1], bv), m, n, d


def _d1():
    g = np.random.default_rng(13)
    A = g.standard_normal((300, 1)).astype(np.float32)
    B = g.standard_normal((200, 1)).astype(np.float32)
    A[::4] = 0.0
    return workloads.dense_to_csr(A), workloads.dense_to_csr(B), 300, 200, 1


def _dense_as_csr():
    A, B = workloads.dense_gaussian(400, 350, 30, seed=14)
    return workloads.dense_to_csr(A), workloads.dense_to_csr(B), 400, 350, 30


def _powerlaw_big():
    # the top coordinates carry ~1e5 entries: tables of 2^17-2^18 slots in
    # the multi-workgroup pipeline, as at the full sparse sizes
    m, n, d = 200_000, 190_000, 20_000
    a = workloads.powerlaw_csr(m, d, 20, 1.5, seed=15, role=0)
    b = workloads.powerlaw_csr(n, d, 20, 1.5, seed=15, role=1)
    return a, b, m, n, d


def _unit_values():
    # 0/1 inputs: every stored value is 1, so the sampler takes a present
    # fourth edge as 1 without loading it; A keeps one value of 2 so that
    # only B is all ones (the flag is B's)
    a, b, m, n, d = _powerlaw()
    av = np.ones_like(a[2])
    av[3] = 2.0
    return (a[0], a[1], av), (b[0], b[1], np.ones_like(b[2])), m, n, d


CASES = {"powerlaw": _powerlaw, "ragged": _ragged, "zeros": _explicit_zeros,
         "d1": _d1, "dense_as_csr": _dense_as_csr, "unit": _unit_values}
# tables and sample streams only
CASES_BIG = {"powerlaw_big": _powerlaw_big}


def make(mad, name):
    a, b, m, n, d = {**CASES, **CASES_BIG}[name]()
    say("case", name, "m n d", m, n, d, "nnz", len(a[1]), len(b[1]))
    gp = mad.Plan.csr(tuple(to_dev(x) for x in a), tuple(to_dev(x) for x in b),
                      m, n, d)
    op = oracle.Plan.csr(a[0], a[1], a[2], m, b[0], b[1], b[2], n, d)
    return gp, op, a, b, m, n, d


def _dense(x, rows, d):
    return workloads.csr_to_dense(x[0], x[1], x[2], rows, d)


@pytest.mark.parametrize("name", list(CASES) + list(CASES_BIG))
def test_norms_and_tables_bitexact(mad_gpu, name):
    gp, op, a, b, m, n, d = make(mad_gpu, name)
    g = gp.norms()
    o = op.norms()
    for x, y in zip(g, o):
        assert np.array_equal(x, y)
    at = np.bincount(a[1], minlength=d)
    bt = np.bincount(b[1], minlength=d)
    ks = {0, d - 1, int(np.argmax(at)), int(np.argmax(bt)), d // 2}
    rows = np.diff(a[0])
    iss = {0, m - 1, int(np.argmax(rows)), int(np.argmin(rows)), m // 2}
    checks = [(0, 0)] + [(1, k) for k in ks] + [(2, k) for k in ks] + \
             [(3, i) for i in iss]
    for which, idx in sorted(checks):
        gthr, galias, gself = gp.table(which, idx)
        othr, oal, oitem, N, live, _ = op.table(which, idx)
        assert np.array_equal(gthr, othr), (which, idx)
        if which == 0 or not live:
            if which == 0:
                assert np.array_equal(galias, oal), (which, idx)
            continue
        assert np.array_equal(galias, oitem[oal]), (which, idx)
        assert np.array_equal(gself[:N], oitem), (which, idx)
    gp.close()


@pytest.mark.parametrize("name", list(CASES) + list(CASES_BIG))
def test_sample_stream_bitexact(mad_gpu, name):
    gp, op, a, b, m, n, d = make(mad_gpu, name)
    s = 200_000
    F = op.fix_exponent(s)
    assert gp.fix_exponent(s) == F
    if op.wnorm <= 0:
        pytest.skip("no weight")
    for l0, cnt in ((0, 6000), (s - 4000, 4000), ((1 << 40) - 64, 64)):
        g = gp.samples(seed=5, l0=l0, count=cnt, F=F)
        o = op.samples(5, l0, cnt, F)
        for key in ("k", "i", "j", "kp", "inc"):
            assert np.array_equal(g[key], o[key]), (key, l0)
    gp.close()


def _c_scale(Ad, Bd, keys, n):
    return (np.abs(Ad[keys // n].astype(np.float64)) *
            np.abs(Bd[keys % n].astype(np.float64))).sum(1)


@pytest.mark.parametrize("name", list(CASES))
def test_topk_scores_candidates_bitexact(mad_gpu, name):
    gp, op, a, b, m, n, d = make(mad_gpu, name)
    Ad, Bd = _dense(a, m, d), _dense(b, n, d)
    for s, tp, t in ((200_000, 300, 10), (30_000, 10**6, 20), (0, 10, 5)):
        say("topk", name, s, tp, t)
        g = gp.topk(t=t, s=s, t_prime=tp, seed=77)
        o = op.topk(seed=77, s=s, t_prime=tp, t=t)
        st = gp.stats()
        assert st["n_pos"] == o["n_pos"] and st["closed"] == o["closed"]
        if s:
            gk, gx, F = gp.scores()
            ok, ox, _ = op.scores(seed=77, s=s, F=o["F"])
            assert F == o["F"]
            assert np.array_equal(gk, ok) and np.array_equal(gx, ox)
        ck, cx, cc = gp.candidates()
        order = np.argsort(o["tp_key"])
        assert np.array_equal(ck, o["tp_key"][order])
        assert np.array_equal(cx, o["tp_x"][order])
        if len(ck):
            err = np.abs(cc.astype(np.float64) - o["tp_c"][order])
            assert np.all(err <= TOL * _c_scale(Ad, Bd, ck, n) + 1e-30)
        gkey = g["i"].cpu().numpy() * n + g["j"].cpu().numpy()
        assert len(gkey) == len(o["key"])
        if not np.array_equal(gkey, o["key"]):
            c64 = (Ad[gkey // n].astype(np.float64) *
                   Bd[gkey % n].astype(np.float64)).sum(1)
            tau = np.abs(o["c"]).min()
            sc = _c_scale(Ad, Bd, gkey, n)
            okeys = set(o["key"].tolist())
            for kk, c, scv in zip(gkey.tolist(), c64.tolist(), sc.tolist()):
                if kk not in okeys:
                    assert abs(abs(c) - tau) <= 2 * TOL * scv
    gp.close()


def test_dense_input_as_csr_matches_dense_plan(mad_gpu):
    A, B = workloads.dense_gaussian(400, 350, 30, seed=14)
    gp, _, a, b, m, n, d = make(mad_gpu, "dense_as_csr")
    dp = mad_gpu.Plan.dense(to_dev(A), to_dev(B))
    F = dp.fix_exponent(50_000)
    g1 = gp.samples(seed=3, l0=0, count=20_000, F=F)
    g2 = dp.samples(seed=3, l0=0, count=20_000, F=F)
    for key in ("k", "i", "j", "kp", "inc"):
        assert np.array_equal(g1[key], g2[key]), key
    gp.close()
    dp.close()


def test_malformed_and_nonfinite_inputs_rejected(mad_gpu):
    a, b, m, n, d = _powerlaw()

    def attempt(a_, b_):
        return mad_gpu.Plan.csr(tuple(to_dev(x) for x in a_),
                                tuple(to_dev(x) for x in b_), m, n, d)

    bad_idx = a[1].copy()
    bad_idx[[40, 41]] = bad_idx[[41, 40]]            # unsorted within a row
    with pytest.raises(mad_gpu.MadError):
        attempt((a[0], bad_idx, a[2]), b)
    oor = b[1].copy()
    oor[5] = d                                       # coordinate out of range
    with pytest.raises(mad_gpu.MadError):
        attempt(a, (b[0], oor, b[2]))
    ptr = a[0].copy()
    ptr[10] = ptr[11] + 1                            # decreasing pointers
    with pytest.raises(mad_gpu.MadError):
        attempt((ptr, a[1], a[2]), b)
    nan = b[2].copy()
    nan[77] = np.nan
    with pytest.raises(mad_gpu.MadError):
        attempt(a, (b[0], b[1], nan))
    # a valid plan still builds after the failures
    gp = attempt(a, b)
    assert gp.stats()["wnorm"] > 0
    gp.close()


def test_unchecked_refresh_regathers_values(mad_gpu):
    """A plan made with MAD_FLAG_NO_CHECK keeps its first build's structure
    (transposes, layouts) and only regathers values on refresh: after new
    values are written into the borrowed arrays, its tables, samples and
    results equal those of a fresh, checked plan on the new values."""
    import torch
    a, b, m, n, d = _powerlaw()
    ta = tuple(to_dev(x) for x in a)
    tb = tuple(to_dev(x) for x in b)
    gp = mad_gpu.Plan.csr(ta, tb, m, n, d, flags=mad_gpu.MAD_FLAG_NO_CHECK)
    gp.topk(t=10, s=50_000, t_prime=300, seed=3)
    g = np.random.default_rng(21)
    av = (g.standard_normal(len(a[2])) * 3).astype(np.float32)
    bv = g.standard_normal(len(b[2])).astype(np.float32)
    ta[2].copy_(torch.from_numpy(av))
    tb[2].copy_(torch.from_numpy(bv))
    torch.cuda.synchronize()
    gp.refresh()
    a2, b2 = (a[0], a[1], av), (b[0], b[1], bv)
    fp = mad_gpu.Plan.csr(tuple(to_dev(x) for x in a2),
                          tuple(to_dev(x) for x in b2), m, n, d)
    for x, y in zip(gp.norms(), fp.norms()):
        assert np.array_equal(x, y)
    for which, idx in ((0, 0), (1, 0), (1, d // 2), (2, 7), (3, 5)):
        for x, y in zip(gp.table(which, idx), fp.table(which, idx)):
            assert np.array_equal(x, y), (which, idx)
    F = fp.fix_exponent(100_000)
    assert gp.fix_exponent(100_000) == F
    g1 = gp.samples(seed=9, l0=0, count=20_000, F=F)
    g2 = fp.samples(seed=9, l0=0, count=20_000, F=F)
    for key in ("k", "i", "j", "kp", "inc"):
        assert np.array_equal(g1[key], g2[key]), key
    r1 = gp.topk(t=20, s=100_000, t_prime=500, seed=4)
    r2 = fp.topk(t=20, s=100_000, t_prime=500, seed=4)
    for k in ("i", "j", "c", "x"):
        assert np.array_equal(r1[k].cpu().numpy(), r2[k].cpu().numpy()), k
    gp.close()
    fp.close()

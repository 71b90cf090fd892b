"""Pins for the oracle's sums, integer quanta, alias tables and the weights of
Alg. 3 (the weights w_ki)."""
import math

import numpy as np
import pytest

import oracle
import workloads

CAP = 1 << 31


# ---------------------------------------------------------------- prefix sums
RUN = oracle.run_length()


def test_prefix_exact_on_small_integers():
    # every partial sum of small integers is exact in FP64, so any order of
    # addition must give the integer cumulative sum
    g = np.random.default_rng(1)
    for N in (1, 2, 63, 64, 65, RUN - 1, RUN, RUN + 1, 1023, 1024, 1025,
              5000, 70001):
        w = g.integers(0, 1000, size=N).astype(np.float64)
        P = oracle.prefix(w)
        assert np.array_equal(P, np.cumsum(w.astype(np.int64)).astype(np.float64))


def test_prefix_run_structure_on_dyadics():
    # 1.0 followed by terms of 2^-60: inside the first run each tiny term is
    # rounded away (half an ulp of 1.0 is 2^-53), but the second run sums its
    # RUN tiny terms on their own (exactly RUN * 2^-60) before the run offset
    # 1.0 is added.  A single left-to-right sum would stay at 1.0.
    R = RUN
    N = 2 * R + R // 2
    w = np.full(N, 2.0 ** -60)
    w[0] = 1.0
    P = oracle.prefix(w)
    assert P[R - 1] == 1.0
    assert P[2 * R - 1] == 1.0 + R * 2.0 ** -60
    assert P[N - 1] == 1.0 + R * 2.0 ** -60 + (N - 2 * R) * 2.0 ** -60


def test_prefix_monotone_and_zero_preserving():
    g = np.random.default_rng(2)
    for N in (1000, 1024, 4097, 30000):
        w = g.lognormal(0, 3, size=N)
        w[g.random(N) < 0.2] = 0.0
        w[::RUN] = 0.0                    # zeros at run starts
        w[RUN - 1::RUN] = 1e-300          # tiny terms at run ends
        P = oracle.prefix(w)
        assert np.all(np.diff(P) >= 0)
        z = np.nonzero(w[1:] == 0)[0] + 1
        assert np.array_equal(P[z], P[z - 1])


def test_prefix_close_to_exact_sum():
    g = np.random.default_rng(3)
    w = g.random(100000)
    P = oracle.prefix(w)
    exact = math.fsum(w)
    # two-level order: error bounded by about (runs + run length) * eps * sum
    runs = -(-len(w) // RUN)
    assert abs(P[-1] - exact) <= (RUN + runs) * 2.3e-16 * exact


# --------------------------------------------------------------------- quanta
@pytest.mark.parametrize("N", [1, 2, 3, 7, 64, 100, 1000, 1025, 4096, 10000])
def test_quanta_sum_and_sign(N):
    g = np.random.default_rng(N)
    w = g.exponential(size=N)
    w[g.random(N) < 0.1] = 0.0
    if not w.any():
        w[0] = 1.0
    q, live = oracle.quanta(w)
    L = oracle.ceil_log2(N)
    assert live
    assert len(q) == 1 << L
    assert int(q.astype(object).sum()) == 1 << (L + 31)
    assert np.all(q[N:] == 0)
    assert np.all(q[:N][w == 0] == 0)


def test_quanta_proportional_to_weights():
    g = np.random.default_rng(5)
    w = g.exponential(size=777)
    q, _ = oracle.quanta(w)
    L = oracle.ceil_log2(777)
    p = q[:777].astype(np.float64) / 2.0 ** (L + 31)
    # each quantum is within one unit (plus the FP64 prefix error) of 2^K w/T
    err = np.abs(p - w / w.sum()) * 2.0 ** (L + 31)
    assert err.max() <= 2.0 + 2.0 ** (L + 31) * 1e-13


def test_quanta_closed_form_on_dyadic_weights():
    # weights that are multiples of a power of two with a power-of-two total:
    # the integer CDF is exact, q_r = w_r * 2^K / T
    w = np.array([1, 3, 0, 4, 8, 0, 0, 16], np.float64)  # T = 32
    q, live = oracle.quanta(w)
    K = 3 + 31
    assert live
    assert [int(x) for x in q] == [int(v) * (1 << K) // 32 for v in w]


def test_quanta_empty_table():
    q, live = oracle.quanta(np.zeros(5))
    assert not live and not q.any()


# -------------------------------------------------------------------- aliases
def induced_quanta(thr, al):
    """What each item receives from an alias table: slot u gives thr[u] coin
    values to u and 2^31 - thr[u] to alias[u]."""
    got = np.zeros(len(thr), dtype=object)
    for u in range(len(thr)):
        got[u] += int(thr[u])
        got[int(al[u])] += CAP - int(thr[u])
    return got


@pytest.mark.parametrize("N", [1, 2, 5, 16, 100, 1000, 1025, 3000])
def test_alias_induces_exact_quanta(N):
    g = np.random.default_rng(10 + N)
    w = g.lognormal(0, 2, size=N)
    w[g.random(N) < 0.15] = 0.0
    if not w.any():
        w[-1] = 1.0
    q, _ = oracle.quanta(w)
    thr, al = oracle.alias(q)
    assert np.all(thr < CAP)
    got = induced_quanta(thr, al)
    assert [int(x) for x in got] == [int(x) for x in q]


def test_alias_special_shapes():
    for q in ([CAP], [2 * CAP, 0], [0, 2 * CAP], [CAP, CAP, CAP, CAP],
              [4 * CAP - 3, 1, 1, 1], [1, 1, 1, 4 * CAP - 3],
              [CAP + 5, CAP - 5, CAP - 1, CAP + 1]):
        q = np.array(q, np.uint64)
        thr, al = oracle.alias(q)
        assert [int(x) for x in induced_quanta(thr, al)] == [int(x) for x in q]


def test_alias_rejects_unbalanced_quanta():
    with pytest.raises(ValueError):
        oracle.alias(np.array([CAP, CAP - 1], np.uint64))


def test_alias_sweep_order_is_canonical():
    # hand-worked sweep: q = [C/2, 3C/2]: light 0 takes C/2 from heavy 1,
    # which keeps exactly C and is full
    thr, al = oracle.alias(np.array([CAP // 2, 3 * CAP // 2], np.uint64))
    assert list(thr) == [CAP // 2, 0] and list(al) == [1, 1]
    # q = [0, C/4, 7C/4, 2C]: light 0 drains heavy 2 to 3C/4 (< C), so slot 2
    # closes with thr 3C/4 and alias 3; light 1 then takes 3C/4 from 3
    q = np.array([0, CAP // 4, 7 * CAP // 4, 2 * CAP], np.uint64)
    thr, al = oracle.alias(q)
    assert list(al) == [2, 3, 3, 3]
    assert list(thr) == [0, CAP // 4, 3 * CAP // 4, 0]


def test_draw_frequencies_match_quanta_exhaustively():
    # enumerate every (slot, coin-class) of a small table
    w = np.array([0.5, 0.0, 2.0, 1.0, 0.25])
    q, _ = oracle.quanta(w)
    thr, al = oracle.alias(q)
    counts = np.zeros(len(q), dtype=object)
    for u in range(len(thr)):
        for coin, mult in ((0, int(thr[u])), (CAP - 1, CAP - int(thr[u]))):
            if mult == 0:
                continue
            U = (u << (64 - 3)) | coin
            counts[oracle.draw(thr, al, U)] += mult
    assert [int(x) for x in counts] == [int(x) for x in q]


# -------------------------------------------------------------------- weights
def test_plan_norms_and_wnorm_closed_form():
    A, B = workloads.tiny(30, 20, 6)
    p = oracle.Plan.dense(A, B)
    na, nb, v, om = p.norms()
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    assert np.allclose(na, np.abs(A64).sum(1), rtol=1e-14)
    assert np.allclose(nb, np.abs(B64).sum(0), rtol=1e-14)
    W = np.abs(A64) * na[:, None] * nb[None, :]      # w_ki of Alg. 3
    assert np.allclose(v, (np.abs(A64) * na[:, None]).sum(0), rtol=1e-14)
    assert np.allclose(om, nb * v, rtol=1e-15)
    assert p.wnorm == pytest.approx(W.sum(), rel=1e-13)


def test_plan_weights_exact_on_integer_inputs():
    # small integer entries: every sum and product is exact
    g = np.random.default_rng(4)
    A = g.integers(-3, 4, size=(12, 5)).astype(np.float32)
    B = g.integers(-3, 4, size=(9, 5)).astype(np.float32)
    p = oracle.Plan.dense(A, B)
    na, nb, v, om = p.norms()
    Ai, Bi = np.abs(A).astype(np.int64), np.abs(B).astype(np.int64)
    assert np.array_equal(na, Ai.sum(1).astype(float))
    assert np.array_equal(nb, Bi.sum(0).astype(float))
    v_int = (Ai * Ai.sum(1)[:, None]).sum(0)
    assert np.array_equal(v, v_int.astype(float))
    assert p.wnorm == float((v_int * Bi.sum(0)).sum())


def test_tables_hold_stage_distributions():
    # each table's induced quanta, divided by 2^K, equals its stage
    # distribution to within 2^-K per item (R2: T0 ~ nb v, T1[k] ~ |a| na,
    # T2[k] ~ |b|, T3[i] ~ |a|)
    A, B = workloads.tiny(9, 7, 4, seed=3)
    p = oracle.Plan.dense(A, B)
    na, nb, v, om = p.norms()
    A64, B64 = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))

    def check(which, idx, w):
        thr, al, item, N, live, tot = p.table(which, idx)
        L = oracle.ceil_log2(N)
        got = induced_quanta(thr, al)
        prob = np.array([float(x) for x in got[:N]]) / 2.0 ** (L + 31)
        assert np.all(np.array([int(x) for x in got[N:]]) == 0)
        assert np.allclose(prob, w / w.sum(), atol=4 * 2.0 ** -(L + 31) + 1e-14)

    check(0, 0, om)
    for k in range(4):
        check(1, k, A64[:, k] * na)
        check(2, k, B64[:, k])
    for i in range(9):
        check(3, i, A64[i])


def test_dense_and_sparse_plans_agree_without_zeros():
    # a dense input with no zero entry is the same set of weights in the
    # sparse form, so every table and every sample must coincide
    A, B = workloads.dense_gaussian(40, 30, 7, seed=5)
    pd = oracle.Plan.dense(A, B)
    ps = oracle.Plan.csr(*workloads.dense_to_csr(A), 40,
                         *workloads.dense_to_csr(B), 30, 7)
    assert pd.wnorm == ps.wnorm
    F = pd.fix_exponent(5000)
    sd = pd.samples(7, 0, 5000, F)
    ss = ps.samples(7, 0, 5000, F)
    for key in ("k", "i", "j", "kp", "inc"):
        assert np.array_equal(sd[key], ss[key])

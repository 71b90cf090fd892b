"""Pins for the oracle's sparse path and its one-query (MIPS) form, checked
against what the paper and the mathematics fix rather than against another
implementation.

The sparse oracle finds a coordinate's value by binary search in a vector's
sorted coordinate list (zero when absent) and builds the per-coordinate
tables from a ragged transpose.  These tests read every expected value from
the densified matrices with numpy indexing instead:

* the tables: each coordinate's table lists exactly the vectors that store
  that coordinate, in ascending order, and induces the stage distribution
  of Alg. 3 (|a_ki| ||a_i||_1 for T1[k], |b_kj| for T2[k], |a_k'i| for
  T3[i]);
* each sample's increment: sgn(a_ki b_kj a_k'i) rne(b_k'j 2^F) with the
  signed fourth edge b_k'j (the score update of Alg. 3), zero exactly when
  b_k'j is zero or absent;
* Lemma 1: the three-path (k', i, k, j) frequencies, by chi-square;
* Lemma 2: E[x_ij] = s c_ij^2 / ||W||_1, by a z-test with the exact
  per-sample variance;
* Alg. 2: with every pair a candidate, the exhaustive answer.

Inputs are ragged: empty vectors, coordinates no vector stores, stored
zeros, and a closure rate well below 100%.
"""
import itertools

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads

CAP = 1 << 31


def tiny_ragged():
    """m = 4, n = 4, d = 5.  a_2 and b_2 are empty, coordinate 4 is stored by
    no vector, b_3 stores an explicit zero at coordinate 1."""
    a = {0: {0: 1.5, 2: -0.75},
         1: {1: 2.0, 2: 0.5, 3: -1.25},
         2: {},
         3: {0: -0.375, 3: 0.875}}
    b = {0: {0: 0.8, 1: -1.2},
         1: {2: 1.7, 3: 0.5},
         2: {},
         3: {0: -0.6, 1: 0.0, 2: 0.3, 3: 1.0}}
    return _to_csr(a, 4), _to_csr(b, 4), 4, 4, 5


def _to_csr(vecs, rows):
    ptr = [0]
    idx, val = [], []
    for r in range(rows):
        for k in sorted(vecs[r]):
            idx.append(k)
            val.append(vecs[r][k])
        ptr.append(len(idx))
    return (np.array(ptr, np.int64), np.array(idx, np.int32),
            np.array(val, np.float32))


def dense_of(csr, rows, d):
    return workloads.csr_to_dense(*csr, rows, d)


def stored_mask(csr, rows, d):
    ptr, idx, _ = csr
    M = np.zeros((rows, d), bool)
    r = np.repeat(np.arange(rows), np.diff(ptr))
    M[r, idx] = True
    return M


def lemma1_probs(A, B):
    """Pr(k', i, k, j) = |a_ki b_kj a_k'i| / ||W||_1 (Lemma 1), dense arrays."""
    A64, B64 = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))
    W = (A64 * A64.sum(1)[:, None] * B64.sum(0)[None, :]).sum()
    P = np.einsum("ik,jk,ip->pikj", A64, B64, A64) / W
    return P, W


def moments(A, B):
    """Exact mean c_ij^2 / W and variance of one sample's increment to x_ij."""
    P, W = lemma1_probs(A, B)
    B64 = B.astype(np.float64)
    C = A.astype(np.float64) @ B64.T
    mean = C ** 2 / W
    m2 = np.einsum("pikj,jp->ij", P, B64 ** 2)
    return mean, m2 - mean ** 2


def csr_plan(a, b, m, n, d):
    return oracle.Plan.csr(*a, m, *b, n, d)


def induced(thr, al):
    got = np.zeros(len(thr), dtype=object)
    for u in range(len(thr)):
        got[u] += int(thr[u])
        got[int(al[u])] += CAP - int(thr[u])
    return got


def test_ragged_tables_list_stored_vectors_with_stage_weights():
    a, b, m, n, d = workloads.ragged_csr(30, 24, 17, seed=3)
    A, B = dense_of(a, m, d), dense_of(b, n, d)
    MA, MB = stored_mask(a, m, d), stored_mask(b, n, d)
    p = csr_plan(a, b, m, n, d)
    A64, B64 = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))
    na = A64.sum(1)
    got_na, got_nb, got_v, _ = p.norms()
    assert np.allclose(got_na, na, rtol=1e-14, atol=0)
    assert np.allclose(got_nb, B64.sum(0), rtol=1e-14, atol=0)
    assert np.allclose(got_v, (A64 * na[:, None]).sum(0), rtol=1e-14, atol=0)

    def check(which, idx, members, w):
        thr, al, item, N, live, tot = p.table(which, idx)
        assert np.array_equal(item, members)  # ascending, stored zeros kept
        assert N == len(members)
        assert live == (w.sum() > 0)
        if not live:
            return
        L = oracle.ceil_log2(N)
        q = induced(thr, al)
        prob = np.array([float(x) for x in q[:N]]) / 2.0 ** (L + 31)
        assert all(int(x) == 0 for x in q[N:])
        assert np.allclose(prob, w / w.sum(), atol=4 * 2.0 ** -(L + 31) + 1e-14)
        assert np.all(prob[w == 0] == 0)  # weight 0 is never drawn

    for k in range(d):
        rows_a = np.nonzero(MA[:, k])[0]
        check(1, k, rows_a, A64[rows_a, k] * na[rows_a])
        rows_b = np.nonzero(MB[:, k])[0]
        check(2, k, rows_b, B64[rows_b, k])
    for i in range(m):
        cols = np.nonzero(MA[i])[0]
        check(3, i, cols, A64[i, cols])


def test_ragged_increments_match_the_densified_inputs():
    a, b, m, n, d = workloads.ragged_csr(60, 50, 40, seed=5)
    A, B = dense_of(a, m, d), dense_of(b, n, d)
    assert (A == 0).all(1).any() and (B == 0).all(1).any()  # empty vectors
    assert ((A == 0).all(0) & (B == 0).all(0)).any()        # empty coordinate
    p = csr_plan(a, b, m, n, d)
    s = 200_000
    F = p.fix_exponent(s)
    assert F == oracle.fix_exponent(float(np.abs(B).max()), s)
    r = p.samples(seed=11, l0=0, count=s, F=F)
    k, i, j, kp = (r[x].astype(np.int64) for x in ("k", "i", "j", "kp"))
    # every drawn entry carries weight: stored zeros and absent entries never
    assert np.all(A[i, k] != 0) and np.all(B[j, k] != 0) and np.all(A[i, kp] != 0)
    v = B[j, kp].astype(np.float64)
    neg = np.signbit(A[i, k]) ^ np.signbit(B[j, k]) ^ np.signbit(A[i, kp])
    fix = np.rint(np.ldexp(v, F)).astype(np.int64)   # signed b_k'j
    want = np.where(neg, -fix, fix)
    want[v == 0] = 0
    assert np.array_equal(r["inc"], want)
    closure = np.count_nonzero(v) / s
    assert r["closed"] == np.count_nonzero(v)
    assert 0.05 < closure < 0.9


def test_ragged_lemma1_three_path_frequencies():
    a, b, m, n, d = tiny_ragged()
    A, B = dense_of(a, m, d), dense_of(b, n, d)
    p = csr_plan(a, b, m, n, d)
    P, W = lemma1_probs(A, B)
    assert p.wnorm == pytest.approx(W, rel=1e-14)
    s = 1_000_000
    r = p.samples(seed=2, l0=0, count=s, F=p.fix_exponent(s))
    flat = ((r["kp"].astype(np.int64) * m + r["i"]) * d + r["k"]) * n + r["j"]
    counts = np.bincount(flat, minlength=P.size).reshape(P.shape)
    keep = P > 0
    assert counts[~keep].sum() == 0
    pval = stats.chisquare(counts[keep], P[keep] * s).pvalue
    assert pval > 1e-4
    # power: the same counts reject a law that ignores the a_i norms
    A64, B64 = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))
    Q = np.einsum("ik,jk,ip->pikj", A64, B64, A64 / np.maximum(A64.sum(1), 1e-300)[:, None])
    Q /= Q.sum()
    assert stats.chisquare(counts[keep], Q[keep] * s).pvalue < 1e-30
    # closure well below 100%: b_k'j is absent for many three-paths
    assert 0.2 < r["closed"] / s < 0.8


def test_ragged_lemma2_expectation():
    a, b, m, n, d = tiny_ragged()
    A, B = dense_of(a, m, d), dense_of(b, n, d)
    p = csr_plan(a, b, m, n, d)
    s = 2_000_000
    F = p.fix_exponent(s)
    keys, xfix, closed = p.scores(seed=9, s=s, F=F)
    x = np.zeros(m * n)
    x[keys] = xfix * 2.0 ** -F
    x = x.reshape(m, n)
    mean, var = moments(A, B)
    live = var > 0
    assert np.all(x[~live] == 0)
    z = (x[live] - s * mean[live]) / np.sqrt(s * var[live])
    assert np.abs(z).max() < 4.5
    # a mistake that drops the sign would move some z far out
    wrong = np.einsum("pikj,jp->ij", lemma1_probs(A, B)[0], np.abs(B.astype(np.float64)))
    zw = (s * wrong[live] - s * mean[live]) / np.sqrt(s * var[live])
    assert np.abs(zw).max() > 50


def test_ragged_topk_equals_exhaustive_when_every_pair_is_a_candidate():
    a, b, m, n, d = workloads.ragged_csr(20, 25, 12, seed=7, density=0.4)
    A, B = dense_of(a, m, d), dense_of(b, n, d)
    p = csr_plan(a, b, m, n, d)
    r = p.topk(seed=1, s=3_000_000, t_prime=m * n, t=6)
    k_ex, c_ex = oracle.exact_topk(A, B, 6)
    assert np.all(np.abs(c_ex) > 0)
    assert np.array_equal(r["key"], k_ex)
    assert np.allclose(r["c"], c_ex, rtol=1e-12)
    # verification of every candidate is the exact dot product
    c = (A[r["tp_key"] // n].astype(np.float64) *
         B[r["tp_key"] % n].astype(np.float64)).sum(1)
    assert np.allclose(r["tp_c"], c, rtol=1e-13, atol=1e-13)


def test_mips_form_lemma2_with_query_word():
    # one query (n = 1) with the counter's query word set, as a batch runs
    # query 77: still an unbiased estimator of s c_i^2 / ||W||_1
    A = workloads.tiny(5, 1, 3, seed=31)[0]
    q = np.array([[0.7, -1.3, 0.0]], np.float32)   # a zero coordinate
    p = oracle.Plan.dense(A, q)
    s = 1_000_000
    F = p.fix_exponent(s)
    keys, xfix, _ = p.scores(seed=4, s=s, F=F, qid=77)
    x = np.zeros(5)
    x[keys] = xfix * 2.0 ** -F       # keys are i * 1 + 0
    mean, var = moments(A, q)
    z = (x - s * mean[:, 0]) / np.sqrt(s * var[:, 0])
    assert np.abs(z).max() < 4.5
    # the query word selects another stream: same law, different draws
    r0 = p.samples(4, 0, 1000, F, qid=0)
    r1 = p.samples(4, 0, 1000, F, qid=77)
    assert not np.array_equal(r0["i"], r1["i"])
    u0 = oracle.philox4x64_10([5, 77, 0, 0], [4, 0])
    u1 = oracle.philox4x64_10([5, 0, 0, 0], [4, 0])
    assert not np.array_equal(u0, u1)


def test_mips_form_matches_general_plan_with_one_vector():
    # replacing B by one query keeps the A-side tables: the stream equals a
    # plan built from scratch on (A, q)
    A, _ = workloads.dense_gaussian(30, 1, 6, seed=4)
    q1 = workloads.dense_gaussian(1, 2, 6, seed=5)[1]
    p = oracle.Plan.dense(A, q1[:1])
    p.set_dense_b(q1[1:2])
    fresh = oracle.Plan.dense(A, q1[1:2])
    F = fresh.fix_exponent(5000)
    a = p.samples(3, 0, 5000, F, qid=9)
    b = fresh.samples(3, 0, 5000, F, qid=9)
    for key in ("k", "i", "j", "kp", "inc"):
        assert np.array_equal(a[key], b[key])
    assert np.all(a["j"] == 0)


@pytest.mark.parametrize("kb", [0, 1, 20, 31])
def test_keyed_exponent_keeps_every_score_in_its_bits(kb):
    # Reading R7 with a kb-bit key beside the score: a signed field of
    # 64 - kb bits holds [-2^(63-kb), 2^(63-kb)).  The largest score s
    # increments can reach is s rne(max|b| 2^F), every sample on one pair
    # with the largest |b|; it must stay within 2^(62-kb).
    for bmax in (1e-3, 0.75, 1.0, 1.5, 2.0, 3.999, 4.0, 1e3):
        p = oracle.Plan.dense(np.ones((1, 1), np.float32),
                              np.full((1, 1), bmax, np.float32))
        for s in (1, 2, 3, 1000, 1024, 1025, 10**5):
            F = p.fix_exponent(s, key_bits=kb)
            assert F == p.fix_exponent(s) - kb
            top = s * np.rint(np.ldexp(np.float64(np.float32(bmax)), F))
            assert top <= 2.0 ** (62 - kb)
        # m = n = d = 1: every sample is the same diamond, x = s * inc
        s = 1000
        F = p.fix_exponent(s, key_bits=kb)
        keys, x, closed = p.scores(seed=3, s=s, F=F)
        inc = int(np.rint(np.ldexp(np.float64(np.float32(bmax)), F)))
        assert closed == s and keys.tolist() == [0]
        assert int(x[0]) == s * inc and abs(int(x[0])) <= 2 ** (62 - kb)
        p.close()

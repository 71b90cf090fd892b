"""Pins for the oracle's postprocessing (Alg. 2), its fixed-point scores and
its exhaustive t-MAD."""
import numpy as np
import pytest

import oracle
import workloads


def test_bruteforce_c_loop_equals_numpy_fp64():
    A, B = workloads.dense_gaussian(60, 70, 9, seed=3)
    k1, c1 = oracle.bruteforce_dense(A, B, 25)
    k2, c2 = oracle.exact_topk(A, B, 25, block=17)
    assert np.array_equal(k1, k2)
    assert np.allclose(c1, c2, rtol=1e-13, atol=1e-13)


def test_bruteforce_tie_break_by_pair_index():
    # equal |c| values (binary inputs make many ties) resolve by i*n + j
    A, B = workloads.binary(10, 8, 6, density=0.5, seed=1)
    keys, cs = oracle.bruteforce_dense(A, B, 30)
    C = (A.astype(np.int64) @ B.astype(np.int64).T).ravel()
    order = np.lexsort((np.arange(C.size), -np.abs(C)))[:30]
    assert np.array_equal(keys, order)
    assert np.array_equal(cs, C[order].astype(float))


def test_topk_equals_exhaustive_when_every_pair_is_a_candidate():
    # with t' = mn and enough samples that every top-t pair has x > 0, Alg. 2
    # returns exactly the exhaustive top-t
    A, B = workloads.planted(25, 30, 6, n_planted=5, seed=2)[:2]
    p = oracle.Plan.dense(A, B)
    r = p.topk(seed=4, s=2_000_000, t_prime=25 * 30, t=10)
    k_ex, c_ex = oracle.exact_topk(A, B, 10)
    assert np.array_equal(r["key"], k_ex)
    assert np.allclose(r["c"], c_ex, rtol=1e-12)


def test_post1_selects_largest_scores_with_tie_break():
    A, B = workloads.dense_gaussian(40, 50, 8, seed=6)
    p = oracle.Plan.dense(A, B)
    s, tp = 30000, 200
    F = p.fix_exponent(s)
    keys, xfix, closed = p.scores(seed=2, s=s, F=F)
    r = p.topk(seed=2, s=s, t_prime=tp, t=20, F=F)
    pos = xfix > 0
    assert r["n_pos"] == pos.sum()
    assert len(keys) <= closed <= s  # nnz(X) <= s
    order = np.lexsort((keys[pos], -xfix[pos]))[:tp]
    assert np.array_equal(r["tp_key"], keys[pos][order])
    assert np.array_equal(r["tp_x"], xfix[pos][order])
    # verification: exact FP64 dot products of the candidates
    n = B.shape[0]
    c = (A[r["tp_key"] // n].astype(np.float64) *
         B[r["tp_key"] % n].astype(np.float64)).sum(1)
    assert np.allclose(r["tp_c"], c, rtol=1e-13, atol=1e-12)
    # final selection: top-t by |c| among the candidates
    o3 = np.lexsort((r["tp_key"], -np.abs(r["tp_c"])))[:20]
    assert np.array_equal(r["key"], r["tp_key"][o3])


def test_fewer_candidates_than_budget():
    A, B = workloads.dense_gaussian(30, 30, 5, seed=7)
    p = oracle.Plan.dense(A, B)
    r = p.topk(seed=1, s=50, t_prime=1000, t=500)
    assert len(r["tp_key"]) == r["n_pos"] <= 50
    assert len(r["key"]) == len(r["tp_key"])


def test_fixed_point_scores_are_exact_sums():
    # x_fix * 2^-F is the exact sum of the sampled increments: compare with
    # an exact rational sum of the per-sample stream
    A, B = workloads.tiny(15, 12, 5, seed=12)
    p = oracle.Plan.dense(A, B)
    s = 20000
    F = p.fix_exponent(s)
    r = p.samples(6, 0, s, F)
    keys, xfix, _ = p.scores(seed=6, s=s, F=F)
    key = r["i"].astype(np.int64) * 12 + r["j"]
    ref = {}
    for kk, inc in zip(key, r["inc"]):
        if inc != 0:
            ref[int(kk)] = ref.get(int(kk), 0) + int(inc)
    assert dict(zip(keys.tolist(), xfix.tolist())) == ref
    # each increment is sgn(a_ki b_kj a_k'i) * b_k'j (the score update of Alg. 3) scaled by
    # 2^F and rounded to the nearest integer (halves to even)
    v = B[r["j"], r["kp"]].astype(np.float64)
    sg = np.sign(A[r["i"], r["k"]]) * np.sign(B[r["j"], r["k"]]) * \
        np.sign(A[r["i"], r["kp"]])
    want = np.where(v != 0, sg * np.rint(np.ldexp(v, F)), 0)
    assert np.array_equal(r["inc"], want.astype(np.int64))


def test_fix_exponent_bounds_the_sum():
    for bmax in (1e-20, 0.3, 1.0, 4.9, 1e20):
        for s in (1, 2, 3, 1000, 10**7, 10**9):
            F = oracle.fix_exponent(bmax, s)
            # |inc| <= bmax * 2^F < 2^(62 - ceil log2 s): s of them fit in int63
            assert np.log2(bmax) + F < 62 - np.ceil(np.log2(max(s, 2))) + 1e-9
            assert np.log2(bmax) + F >= 61 - np.ceil(np.log2(max(s, 2))) - 1e-9


def test_empty_support_gives_no_output():
    A = np.zeros((5, 3), np.float32)
    B = np.ones((4, 3), np.float32)
    p = oracle.Plan.dense(A, B)
    assert p.wnorm == 0.0
    r = p.topk(seed=0, s=1000, t_prime=10, t=5)
    assert len(r["key"]) == 0 and r["n_pos"] == 0


def test_threshold_recall():
    A, B = workloads.dense_gaussian(30, 30, 5, seed=9)
    k, c = oracle.exact_topk(A, B, 10)
    assert oracle.threshold_recall(k, A, B, c, 10) == 1.0
    assert oracle.threshold_recall(k[:5], A, B, c, 10) == 0.5


def test_scores_merged_from_sample_ranges_and_post():
    # X is an exact int64 sum, so sampling [0, s) in ranges and summing each
    # key's increments gives the same X, and Alg. 2 on it the same output
    A, B = workloads.dense_gaussian(60, 45, 7, seed=8)
    p = oracle.Plan.dense(A, B)
    s, tp, t = 50_000, 300, 12
    F = p.fix_exponent(s)
    keys, xfix, _ = p.scores(seed=6, s=s, F=F)
    parts = []
    for l0, cnt in ((0, 7001), (7001, 20000), (27001, 22999)):
        r = p.samples(6, l0, cnt, F)
        closed = r["inc"] != 0
        parts.append((r["i"][closed].astype(np.int64) * 45 + r["j"][closed],
                      r["inc"][closed]))
    mk, mx = oracle.merge_scores(parts)
    assert np.array_equal(mk, keys) and np.array_equal(mx, xfix)
    full = p.topk(seed=6, s=s, t_prime=tp, t=t)
    post = p.post(mk[::-1].copy(), mx[::-1].copy(), tp, t)  # any order
    for k in ("tp_key", "tp_x", "tp_c", "key", "x", "c", "n_pos"):
        assert np.array_equal(post[k], full[k]), k


def test_sparse_exact_topk_equals_dense_definition():
    # the sparse product of the oracle against the plain dense definition
    # on the same (densified) inputs, pairs with c != 0
    a, b, m, n, d = workloads.ragged_csr(70, 90, 30, seed=12, density=0.15)
    A = workloads.csr_to_dense(*a, m, d)
    B = workloads.csr_to_dense(*b, n, d)
    ks, cs = oracle.exact_topk_sparse(a, b, m, n, d, 40)
    kd, cd = oracle.bruteforce_dense(A, B, 40)
    nz = cd != 0
    assert np.array_equal(ks, kd[nz][:len(ks)])
    assert np.allclose(cs, cd[nz][:len(ks)], rtol=1e-13, atol=0)
    assert len(ks) == min(40, int(np.count_nonzero(
        A.astype(np.float64) @ B.astype(np.float64).T)))

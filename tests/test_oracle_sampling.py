"""Statistical and closed-form pins for the oracle's sampler (Alg. 3):
Lemma 1 (three-path probability), Lemma 2 (expectation of x_ij), the binary
diamond count of Sec. 3.1, a one-coordinate closed form and Theorem 4's
separation.  Every check uses fixed seeds, so each outcome is deterministic;
chi-square thresholds are p > 1e-4 (a correct sampler fails one with
probability 1e-4 per seed), while each planted mistake below fails by
orders of magnitude."""
import itertools

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads


def lemma1_probs(A, B):
    """Pr(three-path (k', i, k, j)) = |a_ki b_kj a_k'i| / ||W||_1 (Lemma 1)."""
    A64, B64 = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))
    m, d = A.shape
    n = B.shape[0]
    na = A64.sum(1)
    nb = B64.sum(0)
    W = (A64 * na[:, None] * nb[None, :]).sum()
    P = np.zeros((d, m, d, n))  # [k', i, k, j]
    for kp, i, k, j in itertools.product(range(d), range(m), range(d), range(n)):
        P[kp, i, k, j] = A64[i, k] * B64[j, k] * A64[i, kp] / W
    return P, W


def sample_counts(p, s, seed, shape):
    F = p.fix_exponent(s)
    r = p.samples(seed, 0, s, F)
    d, m, _, n = shape
    flat = ((r["kp"].astype(np.int64) * m + r["i"]) * d + r["k"]) * n + r["j"]
    return np.bincount(flat, minlength=d * m * d * n).reshape(shape), r, F


def chi2_pvalue(counts, probs):
    keep = probs > 0
    assert counts[~keep].sum() == 0  # a zero-probability path is never drawn
    obs = counts[keep].astype(np.float64)
    exp = probs[keep] * counts.sum()
    return stats.chisquare(obs, exp).pvalue


def test_lemma1_three_path_frequencies():
    A, B = workloads.tiny(2, 2, 3, seed=11)
    p = oracle.Plan.dense(A, B)
    P, W = lemma1_probs(A, B)
    assert p.wnorm == pytest.approx(W, rel=1e-14)
    counts, _, _ = sample_counts(p, 1_000_000, seed=5, shape=P.shape)
    assert chi2_pvalue(counts, P) > 1e-4


def test_lemma1_rejects_the_wrong_weight_reading():
    # With the per-coordinate norm ||a_*k||_1 in place of ||a_i||_1 (the
    # other reading of the weight), the three-path law differs; the same
    # samples must reject it, so the chi-square above has power to catch
    # that mistake in the oracle.
    A, B = workloads.tiny(2, 2, 3, seed=11)
    p = oracle.Plan.dense(A, B)
    P, _ = lemma1_probs(A, B)
    counts, _, _ = sample_counts(p, 1_000_000, seed=5, shape=P.shape)
    A64, B64 = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))
    na_wrong = A64.sum(0)  # ||a_*k||_1 indexed by coordinate
    d, m = 3, 2
    Q = np.zeros_like(P)
    for kp, i, k, j in itertools.product(range(d), range(m), range(d), range(2)):
        wki = A64[i, k] * na_wrong[k] * B64[:, k].sum()
        Q[kp, i, k, j] = wki * (B64[j, k] / B64[:, k].sum()) * (A64[i, kp] / A64[i].sum())
    Q /= Q.sum()
    assert chi2_pvalue(counts, Q) < 1e-30


def per_sample_moments(A, B):
    """Exact mean and variance of X_{ij,l} (the per-sample increment of pair
    (i, j)) from Lemma 1: mean c_ij^2 / W, second moment
    sum_{k,k'} Pr(k',i,k,j) b_k'j^2."""
    P, W = lemma1_probs(A, B)
    B64 = B.astype(np.float64)
    C = A.astype(np.float64) @ B64.T
    m, n = C.shape
    mean = C ** 2 / W
    m2 = np.zeros((m, n))
    for i in range(m):
        for j in range(n):
            m2[i, j] = (P[:, i, :, j].sum(axis=1) * B64[j] ** 2).sum()
    return mean, m2 - mean ** 2


def test_lemma2_expectation():
    A, B = workloads.tiny(3, 3, 4, seed=21)
    p = oracle.Plan.dense(A, B)
    s = 2_000_000
    F = p.fix_exponent(s)
    keys, xfix, _ = p.scores(seed=9, s=s, F=F)
    x = np.zeros((3, 3))
    x.ravel()[keys] = xfix * 2.0 ** -F
    mean, var = per_sample_moments(A, B)
    z = (x - s * mean) / np.sqrt(s * var)
    assert np.abs(z).max() < 4.5


def test_lemma2_rejects_a_dropped_sign():
    # if the sign factor of the score update were dropped, E[x_ij/s] would be
    # sum_{k,k'} Pr * |b_k'j|-weighted terms instead of c^2 / W; the z-test
    # separates the two by far more than its threshold
    A, B = workloads.tiny(3, 3, 4, seed=21)
    s = 2_000_000
    P, W = lemma1_probs(A, B)
    B64 = np.abs(B.astype(np.float64))
    mean, var = per_sample_moments(A, B)
    wrong = np.array([[(P[:, i, :, j].sum(axis=1) * B64[j]).sum()
                       for j in range(3)] for i in range(3)])
    z = (s * wrong - s * mean) / np.sqrt(s * var)
    assert np.abs(z).max() > 50


def test_binary_inputs_count_squared_common_neighbours():
    # Sec. 3.1: a pair (i, j) lies in c_ij^2 diamonds; with binary inputs
    # every increment is 1 and x_ij counts closed diamonds, so
    # E[x_ij] = s c_ij^2 / W (Lemma 2) and the counts are multinomial
    A, B = workloads.binary(6, 5, 8, density=0.5, seed=2)
    p = oracle.Plan.dense(A, B)
    s = 400_000
    F = p.fix_exponent(s)
    r = p.samples(3, 0, s, F)
    inc = r["inc"]
    assert set(np.unique(inc)) <= {0, 1 << F}
    C = A.astype(np.int64) @ B.astype(np.int64).T
    W = p.wnorm
    key = r["i"].astype(np.int64) * 5 + r["j"]
    closed = np.bincount(key[inc != 0], minlength=30)
    probs = (C ** 2).ravel() / W
    obs = np.append(closed, s - closed.sum())
    exp = np.append(probs, 1 - probs.sum()) * s
    keep = exp > 0
    assert obs[~keep].sum() == 0
    assert stats.chisquare(obs[keep], exp[keep]).pvalue > 1e-4


def test_one_coordinate_closed_form():
    # d = 1: k = k' = 0, i ~ a_i^2, j ~ |b_j|, every increment is +|b_j|
    A = np.array([[0.5], [-2.0], [1.5]], np.float32)
    B = np.array([[3.0], [-1.0], [0.25], [-2.0]], np.float32)
    p = oracle.Plan.dense(A, B)
    W = (A[:, 0].astype(float) ** 2).sum() * np.abs(B[:, 0]).sum()
    assert p.wnorm == W
    s = 500_000
    F = p.fix_exponent(s)
    r = p.samples(4, 0, s, F)
    assert np.all(r["k"] == 0) and np.all(r["kp"] == 0)
    assert r["closed"] == s  # closure is 100% when B has no zero
    assert np.array_equal(r["inc"], np.ldexp(np.abs(B[r["j"], 0]).astype(np.float64), F).astype(np.int64))
    cnt = np.bincount(r["i"].astype(np.int64) * 4 + r["j"], minlength=12)
    prob = np.outer(A[:, 0] ** 2 / (A[:, 0] ** 2).sum(),
                    np.abs(B[:, 0]) / np.abs(B[:, 0]).sum()).ravel()
    assert stats.chisquare(cnt, prob * s).pvalue > 1e-4


def test_dense_closure_is_complete():
    # Sec. 6 / Table 1: dense inputs close every three-path
    A, B = workloads.dense_gaussian(50, 40, 10, seed=1)
    p = oracle.Plan.dense(A, B)
    r = p.samples(0, 0, 20000, p.fix_exponent(20000))
    assert r["closed"] == 20000


def test_zero_weight_entries_never_drawn():
    A, B = workloads.tiny(20, 15, 6, seed=8)
    A[A < -0.8] = 0.0
    A[3] = 0.0          # a vector with no weight
    B[:, 2] = 0.0       # a coordinate with no weight in B
    p = oracle.Plan.dense(A, B)
    r = p.samples(1, 0, 50000, p.fix_exponent(50000))
    assert np.all(A[r["i"], r["k"]] != 0)
    assert np.all(B[r["j"], r["k"]] != 0)
    assert np.all(A[r["i"], r["kp"]] != 0)
    assert not np.any(r["i"] == 3)
    assert not np.any(r["k"] == 2)
    closed = r["inc"] != 0
    assert np.array_equal(closed, B[r["j"], r["kp"]] != 0)


@pytest.mark.slow
def test_theorem4_separation_nonneg():
    # nonnegative entries <= K = 1 with a few large dot products; at the
    # sample count of Theorem 4 every c > tau outranks every c < tau/4 in x
    # with probability >= 1 - delta; check it over 10 seeds
    g = np.random.default_rng(0)
    m = n = 12
    d = 6
    A = (g.random((m, d)) * 0.2).astype(np.float32)
    B = (g.random((n, d)) * 0.2).astype(np.float32)
    A[0] = 1.0
    B[0] = 1.0
    A[1, :3] = 1.0
    B[1, :3] = 1.0
    C = A.astype(np.float64) @ B.astype(np.float64).T
    tau = 2.9
    delta = 0.1
    p = oracle.Plan.dense(A, B)
    W = p.wnorm
    s = int(np.ceil(12 * 1.0 * W * np.log(2 * m * n / delta) / tau ** 2))
    big = C > tau
    small = C < tau / 4
    assert big.sum() >= 2 and small.sum() > 50
    F = p.fix_exponent(s)
    ok = 0
    for seed in range(10):
        keys, xfix, _ = p.scores(seed=seed, s=s, F=F)
        x = np.zeros(m * n, np.int64)
        x[keys] = xfix
        x = x.reshape(m, n)
        ok += int(x[big].min() > x[small].max())
    assert ok >= 9

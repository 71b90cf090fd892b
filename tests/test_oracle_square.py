"""Pins for the oracle's squared variant (Sec. 3.2.3: B = A, A symmetric,
C = A^2).  Every closed sample adds half of its increment to x_ij and half
to x_kk', then X <- (X + X^T) / 2 and the diagonal is dropped as in the Gram
case.  The oracle adds the full increment to both, so the stored score of a
pair i < j is four times the symmetrised entry.

Pinned by the expectation this update has from Lemma 1 (each update is
unbiased for c^2 / ||W||_1 of its own pair, because A is symmetric), with
the exact per-sample variance from enumerating every three-path; by a
planted mistake (the second update left out) that the same test rejects by
far; by the update count; and by the exhaustive answer of off-diagonal
pairs of A^2 when every pair is a candidate."""
import itertools

import numpy as np
import pytest

import oracle
import workloads


def _square_plan(A):
    p = oracle.Plan.dense(A, A.copy())
    p.set_square(True)
    return p


def _path_moments(A):
    """Per-sample mean and second moment of the stored increment of every
    unordered pair (a, b), a < b: sum over three-paths (k', i, k, j) with
    probability |a_ik a_jk a_ik'| / W of inc * (number of the two updates
    that land on the pair), inc = sgn(a_ik a_jk a_ik') a_jk'."""
    A64 = A.astype(np.float64)
    m = A.shape[0]
    na = np.abs(A64).sum(1)
    nb = np.abs(A64).sum(0)
    W = (np.abs(A64) * na[:, None] * nb[None, :]).sum()
    mean = np.zeros((m, m))
    m2 = np.zeros((m, m))
    for kp, i, k, j in itertools.product(range(m), repeat=4):
        pr = abs(A64[i, k] * A64[j, k] * A64[i, kp]) / W
        if pr == 0.0 or A64[j, kp] == 0.0:
            continue
        inc = np.sign(A64[i, k] * A64[j, k] * A64[i, kp]) * A64[j, kp]
        hits = {}
        for a, b in ((i, j), (k, kp)):
            if a != b:
                key = (min(a, b), max(a, b))
                hits[key] = hits.get(key, 0) + 1
        for (a, b), h in hits.items():
            mean[a, b] += pr * h * inc
            m2[a, b] += pr * (h * inc) ** 2
    return mean, m2, W


def test_square_expectation_and_variance():
    A = workloads.symmetric(4, density=0.7, seed=3)
    assert np.array_equal(A, A.T)
    m = 4
    C = A.astype(np.float64) @ A.astype(np.float64)
    mean, m2, W = _path_moments(A)
    # each update is unbiased for c^2 / W of its own pair: 4 c^2 / W per
    # sample on a < b (two orientations, two updates)
    iu = np.triu_indices(m, 1)
    assert np.allclose(mean[iu], 4 * C[iu] ** 2 / W, rtol=1e-12, atol=1e-15)
    p = _square_plan(A)
    assert p.wnorm == pytest.approx(W, rel=1e-14)
    s = 2_000_000
    F = p.fix_exponent(s)
    assert F == oracle.fix_exponent(float(np.abs(A).max()), 2 * s)
    keys, xfix, _ = p.scores(seed=7, s=s, F=F)
    a, b = keys // m, keys % m
    assert np.all(a < b)
    x = np.zeros((m, m))
    x[a, b] = xfix * 2.0 ** -F
    var = m2 - mean ** 2
    live = (var > 0) & np.triu(np.ones((m, m), bool), 1)
    z = (x[live] - s * mean[live]) / np.sqrt(s * var[live])
    assert np.abs(z).max() < 4.5
    # the second update left out halves the mean: rejected by far
    zw = (x[live] - s * mean[live] / 2) / np.sqrt(s * var[live])
    assert np.abs(zw).max() > 50


def test_square_update_count():
    # every closed sample contributes two updates (minus diagonal ones):
    # the total |stored| mass equals that of the two keys of every sample
    A = workloads.symmetric(12, density=0.5, seed=4, weighted=False)
    m = 12
    p = _square_plan(A)
    s = 100_000
    F = p.fix_exponent(s)
    r = p.samples(5, 0, s, F)
    closed = r["inc"] != 0
    both = np.concatenate([
        np.where(r["i"][closed] != r["j"][closed], r["inc"][closed], 0),
        np.where(r["k"][closed] != r["kp"][closed], r["inc"][closed], 0)])
    keys, xfix, c = p.scores(seed=5, s=s, F=F)
    assert c == np.count_nonzero(closed)
    assert int(xfix.sum()) == int(both.sum())   # 0/1 inputs: no cancellation


def test_square_topk_equals_exhaustive_off_diagonal():
    A = workloads.symmetric(24, density=0.35, seed=5)
    m = 24
    p = _square_plan(A)
    r = p.topk(seed=3, s=2_000_000, t_prime=m * m, t=8)
    C = A.astype(np.float64) @ A.astype(np.float64)
    iu = np.triu_indices(m, 1)
    cv = C[iu]
    order = np.lexsort((iu[0] * m + iu[1], -np.abs(cv)))[:8]
    want = (iu[0] * m + iu[1])[order]
    assert np.array_equal(r["key"], want)
    assert np.allclose(r["c"], cv[order], rtol=1e-12)

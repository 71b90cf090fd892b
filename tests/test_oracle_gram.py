"""Pins for the oracle's Gram variant (Sec. 3.2.2, B = A): X <- (X + X^T)/2
before Alg. 2, kept exact as x_ij + x_ji on the pair i < j, the diagonal
dropped.  Checked by the symmetrised Lemma 2 expectation and by the
conservation of the off-diagonal mass of the plain X from the same
samples."""
import numpy as np

import oracle
import workloads
from test_oracle_sampling import per_sample_moments


def _gram_plan(A):
    p = oracle.Plan.dense(A, A.copy())
    p.set_gram(True)
    return p


def test_gram_symmetrised_expectation():
    A = workloads.tiny(4, 1, 3, seed=31)[0]
    m = A.shape[0]
    s = 2_000_000
    p = _gram_plan(A)
    F = p.fix_exponent(s)
    keys, xfix, _ = p.scores(seed=13, s=s, F=F)
    i, j = keys // m, keys % m
    assert np.all(i < j)                       # canonical, no diagonal
    mean, var = per_sample_moments(A, A.copy())
    m2 = var + mean ** 2
    x = dict(zip(keys.tolist(), (xfix * 2.0 ** -F).tolist()))
    zmax = 0.0
    for a in range(m):
        for b in range(a + 1, m):
            # one sample lands on (a, b) or on (b, a), never both
            ey = mean[a, b] + mean[b, a]
            vy = m2[a, b] + m2[b, a] - ey ** 2
            z = (x.get(a * m + b, 0.0) - s * ey) / np.sqrt(s * vy)
            zmax = max(zmax, abs(z))
    assert zmax < 4.5


def test_gram_conserves_off_diagonal_mass():
    A, _ = workloads.binary(60, 1, 12, density=0.4, seed=32)
    m = A.shape[0]
    s = 200_000
    plain = oracle.Plan.dense(A, A.copy())
    F = plain.fix_exponent(s)
    k1, x1, c1 = plain.scores(seed=4, s=s, F=F)
    off = (k1 // m) != (k1 % m)
    gram = _gram_plan(A)
    k2, x2, c2 = gram.scores(seed=4, s=s, F=F)
    assert c1 == c2                          # the same closed three-paths
    assert int(x2.sum()) == int(x1[off].sum())
    # every unordered pair of X appears once
    pairs = {(min(a, b), max(a, b)) for a, b in zip(k1[off] // m, k1[off] % m)}
    assert len(pairs) == len(k2)


def test_gram_topk_returns_distinct_vectors():
    A, _ = workloads.binary(80, 1, 16, density=0.3, seed=33)
    m = A.shape[0]
    p = _gram_plan(A)
    r = p.topk(seed=2, s=300_000, t_prime=200, t=20)
    i, j = r["key"] // m, r["key"] % m
    assert np.all(i < j)
    c = (A[i].astype(np.float64) * A[j].astype(np.float64)).sum(1)
    assert np.array_equal(c, r["c"])

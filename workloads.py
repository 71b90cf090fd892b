"""Seeded synthetic inputs for the MAD / MIPS workloads.

This module holds only input generation (numpy ``default_rng`` streams keyed
by ``[workload, role]``): no part of the sampling method's arithmetic.  Both
the CPU oracle and the GPU library consume the buffers it returns, so the two
sides never derive inputs from each other.

Workloads (the paper's datasets are not available; these stand in for them):

* ``dense_gaussian``  -- A (m x d), B (n x d) i.i.d. N(0,1) fp32 (the dense
  SVD-factor workload of the experiments, Sec. 6).
* ``planted``         -- dense Gaussian plus planted pairs: for distinct
  (i, j) the vector b_j is moved along a_i so that a_i . b_j equals a chosen
  target (``sigma_mult`` times sqrt(d), random sign, or drawn from a range).
* ``powerlaw_csr``    -- sparse vectors with exactly ``nnz_per_vec`` distinct
  coordinates drawn from a Zipf law over [0, d), lognormal(0,1) magnitudes
  with random signs (the sparse graph / rating workloads of Sec. 6).
* ``mips``            -- a Gaussian database, Gaussian queries and per-query
  sample budgets log-uniform in [s_lo, s_hi] (Sec. 6.5 protocol).
* ``binary`` / ``nonneg`` -- small special inputs for the analysis checks.
"""
from __future__ import annotations

import numpy as np

WORKLOAD_IDS = {
    "dense_gaussian": 1,
    "planted": 2,
    "powerlaw_csr": 3,
    "planted_wide": 4,
    "mips": 5,
    "binary": 6,
    "nonneg": 7,
    "tiny": 8,
    "ragged_csr": 9,
    "symmetric": 10,
}


def rng(workload: str, role: int, seed: int = 0) -> np.random.Generator:
    return np.random.default_rng([WORKLOAD_IDS[workload], role, seed])


def dense_gaussian(m: int, n: int, d: int, seed: int = 0):
    A = rng("dense_gaussian", 0, seed).standard_normal((m, d), dtype=np.float32)
    B = rng("dense_gaussian", 1, seed).standard_normal((n, d), dtype=np.float32)
    return A, B


def planted(m: int, n: int, d: int, n_planted: int, seed: int = 0,
            sigma_mult: float | tuple[float, float] = 5.0,
            workload: str = "planted"):
    """Gaussian A, B with ``n_planted`` pairs (i_p, j_p), all i_p distinct and
    all j_p distinct, set to a_i . b_j = +-sigma_mult * sqrt(d) (or a value
    drawn uniformly from the range ``sigma_mult`` = (lo, hi))."""
    A = rng(workload, 0, seed).standard_normal((m, d), dtype=np.float32)
    B = rng(workload, 1, seed).standard_normal((n, d), dtype=np.float32)
    g = rng(workload, 2, seed)
    ii = g.choice(m, size=n_planted, replace=False)
    jj = g.choice(n, size=n_planted, replace=False)
    sign = np.where(g.random(n_planted) < 0.5, -1.0, 1.0)
    if isinstance(sigma_mult, tuple):
        mult = g.uniform(sigma_mult[0], sigma_mult[1], size=n_planted)
    else:
        mult = np.full(n_planted, float(sigma_mult))
    target = sign * mult * np.sqrt(d)
    for p in range(n_planted):
        a = A[ii[p]].astype(np.float64)
        b = B[jj[p]].astype(np.float64)
        lam = (target[p] - a @ b) / (a @ a)
        B[jj[p]] = (b + lam * a).astype(np.float32)
    return A, B, ii.astype(np.int64), jj.astype(np.int64)


def powerlaw_csr(rows: int, d: int, nnz_per_vec: int, zipf_a: float = 1.5,
                 seed: int = 0, role: int = 0):
    """CSR (ptr int64, idx int32 ascending, val float32) of ``rows`` vectors,
    each with exactly ``nnz_per_vec`` distinct coordinates.  Coordinates are
    Zipf(zipf_a) ranks 1..d mapped through a fixed random permutation of
    [0, d): each vector keeps the first nnz_per_vec distinct draws of rank
    <= d, in draw order (draws above d and repeats are rejected).
    Magnitudes lognormal(0,1), signs +-1 with probability 1/2."""
    g = rng("powerlaw_csr", role, seed)
    perm = rng("powerlaw_csr", 100, seed).permutation(d).astype(np.int32)
    z = nnz_per_vec
    assert z <= d
    idx = np.empty((rows, z), np.int64)
    todo = np.arange(rows)
    draws = np.zeros((rows, 0), np.int64)
    K = 4 * z
    while todo.size:
        new = g.zipf(zipf_a, size=(todo.size, K)).astype(np.int64)
        D = np.concatenate([draws, new], axis=1) if draws.shape[1] else new
        width = D.shape[1]
        valid = D <= d
        # rejected draws get distinct sentinels above d
        key = np.where(valid, D, d + 1 + np.arange(width)[None, :])
        order = np.argsort(key, axis=1, kind="stable")
        ks = np.take_along_axis(key, order, axis=1)
        first = np.ones_like(ks, dtype=bool)
        first[:, 1:] = ks[:, 1:] != ks[:, :-1]
        keep_sorted = first & (ks <= d)
        keep = np.zeros_like(keep_sorted)
        np.put_along_axis(keep, order, keep_sorted, axis=1)
        take = keep & (np.cumsum(keep, axis=1) <= z)
        done = take.sum(axis=1) == z
        rows_done = todo[done]
        idx[rows_done] = D[done][take[done]].reshape(-1, z) - 1
        todo = todo[~done]
        draws = D[~done]
    idx = perm[idx]
    idx.sort(axis=1)
    val = g.lognormal(0.0, 1.0, size=(rows, z)).astype(np.float32)
    val *= np.where(g.random((rows, z)) < 0.5, -1.0, 1.0).astype(np.float32)
    ptr = np.arange(rows + 1, dtype=np.int64) * z
    return ptr, idx.astype(np.int32).ravel(), val.ravel()


def ragged_csr(m: int, n: int, d: int, seed: int = 0, density: float = 0.2):
    """Small ragged sparse inputs for the sparse-path checks: A (m vectors)
    and B (n vectors) as CSR over d coordinates, each entry stored with
    probability ``density``, N(0,1) values.  The first vector of each side
    is empty, the last coordinate is stored by no vector of either side,
    and about one stored entry in ten is an explicit zero.  Returns
    (a_csr, b_csr, m, n, d)."""
    out = []
    for role, rows in ((0, m), (1, n)):
        g = rng("ragged_csr", role, seed)
        mask = g.random((rows, d)) < density
        mask[0] = False
        mask[:, d - 1] = False
        X = g.standard_normal((rows, d)).astype(np.float32)
        zero = mask & (g.random((rows, d)) < 0.1)
        X[~mask] = 0.0
        X[zero] = 0.0
        ptr = np.zeros(rows + 1, np.int64)
        ptr[1:] = np.cumsum(mask.sum(axis=1))
        r, c = np.nonzero(mask)
        out.append((ptr, c.astype(np.int32), X[r, c].astype(np.float32)))
    return out[0], out[1], m, n, d


def symmetric(m: int, density: float = 0.3, seed: int = 0,
              weighted: bool = True):
    """A symmetric m x m matrix (an undirected graph's adjacency, as in the
    A^2 link-prediction workload of Sec. 6): each pair i <= j is an edge with
    probability ``density``; weights N(0,1) (or 1 when not weighted)."""
    g = rng("symmetric", 0, seed)
    upper = np.triu(g.random((m, m)) < density)
    if weighted:
        W = g.standard_normal((m, m)).astype(np.float32)
    else:
        W = np.ones((m, m), np.float32)
    A = np.where(upper, W, np.float32(0.0))
    A = np.triu(A) + np.triu(A, 1).T
    return np.ascontiguousarray(A, dtype=np.float32)


def csr_to_dense(ptr, idx, val, rows: int, d: int) -> np.ndarray:
    X = np.zeros((rows, d), np.float32)
    r = np.repeat(np.arange(rows), np.diff(ptr))
    X[r, idx] = val
    return X


def dense_to_csr(X: np.ndarray):
    rows, d = X.shape
    nz = X != 0
    ptr = np.zeros(rows + 1, np.int64)
    ptr[1:] = np.cumsum(nz.sum(axis=1))
    r, c = np.nonzero(nz)
    return ptr, c.astype(np.int32), X[r, c].astype(np.float32)


def mips(m: int, d: int, nq: int, s_lo: float = 1e3, s_hi: float = 1e5,
         seed: int = 0):
    A = rng("mips", 0, seed).standard_normal((m, d), dtype=np.float32)
    Q = rng("mips", 1, seed).standard_normal((nq, d), dtype=np.float32)
    e = rng("mips", 2, seed).uniform(np.log10(s_lo), np.log10(s_hi), size=nq)
    s_q = np.round(10.0 ** e).astype(np.int64)
    return A, Q, s_q


def binary(m: int, n: int, d: int, density: float, seed: int = 0):
    A = (rng("binary", 0, seed).random((m, d)) < density).astype(np.float32)
    B = (rng("binary", 1, seed).random((n, d)) < density).astype(np.float32)
    return A, B


def nonneg(m: int, n: int, d: int, seed: int = 0):
    A = rng("nonneg", 0, seed).random((m, d), dtype=np.float32)
    B = rng("nonneg", 1, seed).random((n, d), dtype=np.float32)
    return A, B


def tiny(m: int, n: int, d: int, seed: int = 0):
    """Small signed inputs with a few exact zeros."""
    g = rng("tiny", 0, seed)
    A = g.standard_normal((m, d)).astype(np.float32)
    B = g.standard_normal((n, d)).astype(np.float32)
    return A, B


# -------------------------------------------------------------------------
# the named configurations
# -------------------------------------------------------------------------
CONFIGS = {
    "C1": dict(kind="dense", m=1000, n=1000, d=64, s=100_000, t_prime=100,
               t=10),
    "C2": dict(kind="planted", m=100_000, n=100_000, d=100, n_planted=50,
               sigma=5.0, s=10_000_000, t_prime=10_000, t=100),
    "C3": dict(kind="csr", m=1_000_000, n=1_000_000, d=100_000, nnz=20,
               zipf=1.5, s=100_000_000, t_prime=100_000, t=1000),
    "C4": dict(kind="planted_wide", m=100_000, n=1_000_000, d=256,
               n_planted=1000, sigma=(8.0, 10.0), s=1_000_000_000,
               t_prime=200_000, t=1000),
    "C5": dict(kind="mips", m=1_000_000, d=128, nq=4096, s_lo=1e3, s_hi=1e5,
               t=10),
}


def make(name: str, seed: int = 0, scale: float = 1.0):
    """Inputs of a named configuration.  ``scale`` < 1 shrinks the vector
    counts (not d) for quick runs; the full sizes use scale = 1."""
    cfg = dict(CONFIGS[name])
    sc = lambda v: max(1, int(round(v * scale)))
    if cfg["kind"] == "dense":
        A, B = dense_gaussian(sc(cfg["m"]), sc(cfg["n"]), cfg["d"], seed)
        return cfg, dict(A=A, B=B)
    if cfg["kind"] in ("planted", "planted_wide"):
        A, B, ii, jj = planted(sc(cfg["m"]), sc(cfg["n"]), cfg["d"],
                               min(cfg["n_planted"], sc(cfg["m"]),
                                   sc(cfg["n"])), seed, cfg["sigma"],
                               workload=cfg["kind"])
        return cfg, dict(A=A, B=B, planted_i=ii, planted_j=jj)
    if cfg["kind"] == "csr":
        m, n = sc(cfg["m"]), sc(cfg["n"])
        a = powerlaw_csr(m, cfg["d"], cfg["nnz"], cfg["zipf"], seed, role=0)
        b = powerlaw_csr(n, cfg["d"], cfg["nnz"], cfg["zipf"], seed, role=1)
        return cfg, dict(a=a, b=b, m=m, n=n)
    if cfg["kind"] == "mips":
        A, Q, s_q = mips(sc(cfg["m"]), cfg["d"], sc(cfg["nq"]), cfg["s_lo"],
                         cfg["s_hi"], seed)
        return cfg, dict(A=A, Q=Q, s_q=s_q)
    raise KeyError(name)

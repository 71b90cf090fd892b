"""CPU oracle for diamond sampling (Alg. 3 with Alg. 2) and exhaustive t-MAD.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use this package; the product library
never does.  It shares no code with the GPU path.

The arithmetic lives in ``mad_oracle.c`` (plain C, FP64, single thread); this
module compiles it with gcc on first use and wraps it with ctypes.  The
readings it takes where the paper is silent are listed at the top of the C
file (R1..R8).  ``exact_topk`` is the plain definition of t-MAD
(Definition 1) evaluated with numpy FP64 matrix products.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mad_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
           "-shared", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = False) -> str:
    """Compile the oracle (gcc) into oracle/liboracle.so and return its path."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _declare(_lib)
    return _lib


_i64, _u64, _i32, _dbl = C.c_int64, C.c_uint64, C.c_int32, C.c_double
_P = C.c_void_p


def _declare(L):
    L.orc_philox4x64_10.argtypes = [_P, _P, _P]
    L.orc_prefix.argtypes = [_P, _i64, _P]
    L.orc_plan_set_gram.argtypes = [_P, C.c_int]
    L.orc_plan_set_gram.restype = None
    L.orc_plan_set_square.argtypes = [_P, C.c_int]
    L.orc_plan_set_square.restype = None
    L.orc_run_length.argtypes = []
    L.orc_run_length.restype = C.c_int
    L.orc_quanta.argtypes = [_P, _i64, _P]
    L.orc_quanta.restype = C.c_int
    L.orc_alias.argtypes = [_P, C.c_int, _P, _P]
    L.orc_alias.restype = C.c_int
    L.orc_draw.argtypes = [_P, _P, C.c_int, _u64]
    L.orc_draw.restype = _i64
    L.orc_plan_dense.argtypes = [_P, _i64, _P, _i64, _i64]
    L.orc_plan_dense.restype = _P
    L.orc_plan_csr.argtypes = [_P, _P, _P, _i64, _P, _P, _P, _i64, _i64]
    L.orc_plan_csr.restype = _P
    L.orc_plan_set_dense_b.argtypes = [_P, _P, _i64]
    L.orc_plan_free.argtypes = [_P]
    L.orc_plan_wnorm.argtypes = [_P]
    L.orc_plan_wnorm.restype = _dbl
    L.orc_plan_norms.argtypes = [_P, _P, _P, _P, _P]
    L.orc_plan_table.argtypes = [_P, C.c_int, _i64, _P, _P, _P, _P, _P, _P]
    L.orc_plan_table.restype = _i64
    L.orc_fix_exponent.argtypes = [C.c_float, _i64]
    L.orc_fix_exponent.restype = C.c_int
    L.orc_plan_fix_exponent.argtypes = [_P, _i64]
    L.orc_plan_fix_exponent.restype = C.c_int
    L.orc_plan_fix_exponent_keyed.argtypes = [_P, _i64, C.c_int]
    L.orc_plan_fix_exponent_keyed.restype = C.c_int
    L.orc_plan_samples.argtypes = [_P, _u64, _u64, _i64, _i64, C.c_int,
                                   _P, _P, _P, _P, _P]
    L.orc_plan_samples.restype = _i64
    L.orc_plan_scores.argtypes = [_P, _u64, _u64, _i64, C.c_int, _P, _P,
                                  _i64, _P]
    L.orc_plan_scores.restype = _i64
    L.orc_plan_topk.argtypes = [_P, _u64, _u64, _i64, _i64, _i64, C.c_int,
                                _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_plan_topk.restype = _i64
    L.orc_plan_post.argtypes = [_P, _P, _P, _i64, _i64, _i64, _P, _P, _P, _P,
                                _P, _P, _P, _P]
    L.orc_plan_post.restype = _i64
    L.orc_bruteforce_dense.argtypes = [_P, _i64, _P, _i64, _i64, _i64, _P, _P]
    L.orc_bruteforce_dense.restype = _i64


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------
def philox4x64_10(ctr, key) -> np.ndarray:
    """One Philox4x64-10 block for a 4-word counter and a 2-word key."""
    c = np.asarray(ctr, dtype=np.uint64).reshape(4)
    k = np.asarray(key, dtype=np.uint64).reshape(2)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def run_length() -> int:
    """Run length of the two-level summation order (reading R3)."""
    return int(lib().orc_run_length())


def prefix(w) -> np.ndarray:
    """Two-level run-ordered inclusive prefix sum (reading R3)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    P = np.zeros(len(w), np.float64)
    lib().orc_prefix(_ptr(w), len(w), _ptr(P))
    return P


def ceil_log2(N: int) -> int:
    L = 0
    while (1 << L) < N:
        L += 1
    return L


def quanta(w):
    """Integer quanta q (2^L entries summing to 2^(L+31)); (q, live)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    L = ceil_log2(len(w))
    q = np.zeros(1 << L, np.uint64)
    live = lib().orc_quanta(_ptr(w), len(w), _ptr(q))
    return q, bool(live)


def alias(q):
    """Canonical alias sweep over quanta q (length 2^L); (thr, alias)."""
    q = np.ascontiguousarray(q, dtype=np.uint64)
    L = ceil_log2(len(q))
    assert len(q) == 1 << L
    thr = np.zeros(len(q), np.uint32)
    al = np.zeros(len(q), np.uint32)
    rc = lib().orc_alias(_ptr(q), L, _ptr(thr), _ptr(al))
    if rc != 0:
        raise ValueError("quanta do not sum to 2^(L+31)")
    return thr, al


def draw(thr, al, U: int) -> int:
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    al = np.ascontiguousarray(al, dtype=np.uint32)
    return lib().orc_draw(_ptr(thr), _ptr(al), ceil_log2(len(thr)), int(U))


def fix_exponent(bmax: float, s: int) -> int:
    """Fixed-point exponent F of the score increments (reading R7)."""
    return lib().orc_fix_exponent(float(bmax), int(s))


# --------------------------------------------------------------------------
# plans
# --------------------------------------------------------------------------
class Plan:
    """Tables for the weights w_ki of Alg. 3, for one (A, B); see the C file's
    header."""

    def __init__(self, handle, m, n, d, keep):
        self._h = handle
        self.m, self.n, self.d = m, n, d
        self._keep = keep

    @classmethod
    def dense(cls, A: np.ndarray, B: np.ndarray) -> "Plan":
        A = np.ascontiguousarray(A, dtype=np.float32)
        B = np.ascontiguousarray(B, dtype=np.float32)
        m, d = A.shape
        n, d2 = B.shape
        assert d == d2
        h = lib().orc_plan_dense(_ptr(A), m, _ptr(B), n, d)
        return cls(h, m, n, d, (A, B))

    @classmethod
    def csr(cls, a_ptr, a_idx, a_val, m, b_ptr, b_idx, b_val, n, d) -> "Plan":
        arrs = [np.ascontiguousarray(a_ptr, np.int64),
                np.ascontiguousarray(a_idx, np.int32),
                np.ascontiguousarray(a_val, np.float32),
                np.ascontiguousarray(b_ptr, np.int64),
                np.ascontiguousarray(b_idx, np.int32),
                np.ascontiguousarray(b_val, np.float32)]
        h = lib().orc_plan_csr(_ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]), m,
                               _ptr(arrs[3]), _ptr(arrs[4]), _ptr(arrs[5]), n,
                               d)
        return cls(h, m, n, d, arrs)

    def set_dense_b(self, B: np.ndarray):
        B = np.ascontiguousarray(B, dtype=np.float32)
        n, d = B.shape
        assert d == self.d
        lib().orc_plan_set_dense_b(self._h, _ptr(B), n)
        self.n = n
        self._keep = (self._keep[0], B) if len(self._keep) == 2 else self._keep

    def set_gram(self, gram: bool = True):
        """B = A: X <- (X + X^T) / 2 before Alg. 2 (kept as x_ij + x_ji
        on i < j), diagonal dropped (Sec. 3.2.2)."""
        lib().orc_plan_set_gram(self._h, 1 if gram else 0)

    def set_square(self, square: bool = True):
        """B = A symmetric (C = A^2): each closed sample also updates
        x_kk' (Sec. 3.2.3), then X is symmetrised as for set_gram; the
        stored score of i < j is four times the symmetrised entry and F is
        taken for 2s updates."""
        lib().orc_plan_set_square(self._h, 1 if square else 0)

    def close(self):
        if self._h:
            lib().orc_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def wnorm(self) -> float:
        """||W||_1 (total of the stage-0 table)."""
        return lib().orc_plan_wnorm(self._h)

    def norms(self):
        na = np.zeros(self.m, np.float64)
        nb = np.zeros(self.d, np.float64)
        v = np.zeros(self.d, np.float64)
        om = np.zeros(self.d, np.float64)
        lib().orc_plan_norms(self._h, _ptr(na), _ptr(nb), _ptr(v), _ptr(om))
        return na, nb, v, om

    def table(self, which: int, idx: int = 0):
        """(thr, alias, item, N, live, total) of T0 / T1[idx] / T2[idx] / T3[idx]."""
        L = lib()
        Np = L.orc_plan_table(self._h, which, idx, None, None, None, None,
                              None, None)
        if Np < 0:
            raise IndexError("bad table index")
        thr = np.zeros(Np, np.uint32)
        al = np.zeros(Np, np.uint32)
        N = C.c_int64()
        live = C.c_int32()
        tot = C.c_double()
        L.orc_plan_table(self._h, which, idx, _ptr(thr), _ptr(al), None,
                         C.byref(N), C.byref(live), C.byref(tot))
        item = np.zeros(max(N.value, 1), np.int32)
        L.orc_plan_table(self._h, which, idx, None, None, _ptr(item), None,
                         None, None)
        return thr, al, item[:N.value], N.value, bool(live.value), tot.value

    def fix_exponent(self, s: int, key_bits: int = 0) -> int:
        """F of reading R7; key_bits > 0: a score that shares its 64-bit
        word with a key of that many bits."""
        if key_bits:
            return lib().orc_plan_fix_exponent_keyed(self._h, int(s),
                                                     int(key_bits))
        return lib().orc_plan_fix_exponent(self._h, int(s))

    def samples(self, seed: int, l0: int, count: int, F: int, qid: int = 0):
        """Per-sample stream: dict of k, i, j, kp (int32) and inc (int64)."""
        k = np.zeros(count, np.int32)
        i = np.zeros(count, np.int32)
        j = np.zeros(count, np.int32)
        kp = np.zeros(count, np.int32)
        inc = np.zeros(count, np.int64)
        closed = lib().orc_plan_samples(self._h, seed, qid, l0, count, F,
                                        _ptr(k), _ptr(i), _ptr(j), _ptr(kp),
                                        _ptr(inc))
        return dict(k=k, i=i, j=j, kp=kp, inc=inc, closed=closed)

    def scores(self, seed: int, s: int, F: int, qid: int = 0):
        """Sorted (key, x_fix) of every pair with a closed diamond."""
        cap = max(2 * int(s), 1)
        keys = np.zeros(cap, np.int64)
        x = np.zeros(cap, np.int64)
        closed = C.c_int64()
        nd = lib().orc_plan_scores(self._h, seed, qid, s, F, _ptr(keys),
                                   _ptr(x), cap, C.byref(closed))
        return keys[:nd], x[:nd], closed.value

    def topk(self, seed: int, s: int, t_prime: int, t: int, F: int | None = None,
             qid: int = 0):
        """Alg. 3 with Alg. 2.  Returns a dict with Omega_{t'} (candidate selection order) and
        Omega_t (final selection order) as key / x_fix / c arrays."""
        if F is None:
            F = self.fix_exponent(s)
        tp_key = np.zeros(max(t_prime, 1), np.int64)
        tp_x = np.zeros(max(t_prime, 1), np.int64)
        tp_c = np.zeros(max(t_prime, 1), np.float64)
        t_key = np.zeros(max(t, 1), np.int64)
        t_x = np.zeros(max(t, 1), np.int64)
        t_c = np.zeros(max(t, 1), np.float64)
        ntp = C.c_int64()
        npos = C.c_int64()
        closed = C.c_int64()
        nt = lib().orc_plan_topk(self._h, seed, qid, s, t_prime, t, F,
                                 _ptr(tp_key), _ptr(tp_x), _ptr(tp_c),
                                 C.byref(ntp), _ptr(t_key), _ptr(t_x),
                                 _ptr(t_c), C.byref(npos), C.byref(closed))
        n_tp = ntp.value
        return dict(F=F, tp_key=tp_key[:n_tp], tp_x=tp_x[:n_tp],
                    tp_c=tp_c[:n_tp], key=t_key[:nt], x=t_x[:nt],
                    c=t_c[:nt], n_pos=npos.value, closed=closed.value)


    def post(self, keys, xfix, t_prime: int, t: int):
        """Alg. 2 on a given score matrix X (keys i*n + j, int64 x_fix, any
        order): the same outputs as ``topk`` without its sampling."""
        keys = np.ascontiguousarray(keys, dtype=np.int64)
        xfix = np.ascontiguousarray(xfix, dtype=np.int64)
        tp_key = np.zeros(max(t_prime, 1), np.int64)
        tp_x = np.zeros(max(t_prime, 1), np.int64)
        tp_c = np.zeros(max(t_prime, 1), np.float64)
        t_key = np.zeros(max(t, 1), np.int64)
        t_x = np.zeros(max(t, 1), np.int64)
        t_c = np.zeros(max(t, 1), np.float64)
        ntp = C.c_int64()
        npos = C.c_int64()
        nt = lib().orc_plan_post(self._h, _ptr(keys), _ptr(xfix), len(keys),
                                 t_prime, t, _ptr(tp_key), _ptr(tp_x),
                                 _ptr(tp_c), C.byref(ntp), _ptr(t_key),
                                 _ptr(t_x), _ptr(t_c), C.byref(npos))
        n_tp = ntp.value
        return dict(tp_key=tp_key[:n_tp], tp_x=tp_x[:n_tp], tp_c=tp_c[:n_tp],
                    key=t_key[:nt], x=t_x[:nt], c=t_c[:nt],
                    n_pos=npos.value)


def merge_scores(parts):
    """X from per-range sample streams: concatenate the (key, inc) pairs of
    closed samples and sum each key's increments (exact int64 sums, so the
    split into ranges does not matter)."""
    keys = np.concatenate([p[0] for p in parts]) if parts else \
        np.zeros(0, np.int64)
    inc = np.concatenate([p[1] for p in parts]) if parts else \
        np.zeros(0, np.int64)
    order = np.argsort(keys, kind="stable")
    keys, inc = keys[order], inc[order]
    if len(keys) == 0:
        return keys, inc
    first = np.ones(len(keys), bool)
    first[1:] = keys[1:] != keys[:-1]
    starts = np.nonzero(first)[0]
    return keys[starts], np.add.reduceat(inc, starts)


# --------------------------------------------------------------------------
# exhaustive t-MAD (Definition 1)
# --------------------------------------------------------------------------
def bruteforce_dense(A: np.ndarray, B: np.ndarray, t: int):
    """Plain C loops: every pair in FP64; (keys, c) top-t by |c| then key."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    m, d = A.shape
    n = B.shape[0]
    keys = np.zeros(t, np.int64)
    cs = np.zeros(t, np.float64)
    cnt = lib().orc_bruteforce_dense(_ptr(A), m, _ptr(B), n, d, t, _ptr(keys),
                                     _ptr(cs))
    return keys[:cnt], cs[:cnt]


def exact_topk(A: np.ndarray, B: np.ndarray, t: int, block: int = 4096):
    """t-MAD by numpy FP64 products in row blocks of A: (keys, c) sorted by
    |c| descending then key ascending.  Keeps O(block * n + t) memory."""
    A64 = np.asarray(A, dtype=np.float64)
    B64T = np.ascontiguousarray(np.asarray(B, dtype=np.float64).T)
    m, n = A64.shape[0], B64T.shape[1]
    best_k = np.zeros(0, np.int64)
    best_c = np.zeros(0, np.float64)
    for i0 in range(0, m, block):
        Cb = A64[i0:i0 + block] @ B64T
        flat = np.abs(Cb).ravel()
        take = min(t, flat.size)
        # keep every entry tied with the take-th largest so ties resolve by key
        thr = np.partition(flat, flat.size - take)[flat.size - take]
        sel = np.nonzero(flat >= thr)[0]
        keys = (i0 + sel // n) * n + sel % n
        best_k = np.concatenate([best_k, keys.astype(np.int64)])
        best_c = np.concatenate([best_c, Cb.ravel()[sel]])
        order = np.lexsort((best_k, -np.abs(best_c)))[:t]
        best_k, best_c = best_k[order], best_c[order]
    return best_k, best_c


def exact_topk_sparse(a, b, m: int, n: int, d: int, t: int):
    """t-MAD of sparse inputs (Definition 1) restricted to the pairs with
    c != 0: C = A B^T as a sparse FP64 product (scipy), then the top t by
    |c| descending, key i*n + j ascending.  a, b = (ptr, idx, val)."""
    import scipy.sparse as sp
    A = sp.csr_matrix((np.asarray(a[2], np.float64), np.asarray(a[1]),
                       np.asarray(a[0])), shape=(m, d))
    B = sp.csr_matrix((np.asarray(b[2], np.float64), np.asarray(b[1]),
                       np.asarray(b[0])), shape=(n, d))
    Cm = (A @ B.T).tocoo()
    keep = Cm.data != 0
    keys = Cm.row[keep].astype(np.int64) * n + Cm.col[keep].astype(np.int64)
    c = Cm.data[keep]
    order = np.lexsort((keys, -np.abs(c)))[:t]
    return keys[order], c[order]


def threshold_recall(found_keys, A, B, exact_c, t: int) -> float:
    """Recall by threshold: the fraction of t whose exact |c| reaches the
    exact t-th largest |c| (every correct answer under ties scores 1)."""
    if t == 0:
        return 1.0
    tau = np.sort(np.abs(exact_c))[::-1][t - 1]
    A64 = np.asarray(A, dtype=np.float64)
    B64 = np.asarray(B, dtype=np.float64)
    n = B64.shape[0]
    keys = np.asarray(found_keys, dtype=np.int64)
    if keys.size == 0:
        return 0.0
    c = np.einsum("ij,ij->i", A64[keys // n], B64[keys % n])
    return float(np.count_nonzero(np.abs(c) >= tau)) / t

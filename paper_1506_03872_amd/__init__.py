"""Python binding of libmad.so (include/mad.h): diamond sampling for MAD
search on one MI355X.

Argument marshalling only: every step runs in the HIP library.  Tensors are
torch CUDA (ROCm) tensors; the current torch stream is passed to the
library.  Importing this module does not need a GPU, but loading the library
does need the built ``libmad.so``: call ``paper_1506_03872_amd.build.build()``
first.  There is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmad.so")

MAD_OK, MAD_EINVAL, MAD_ENOMEM, MAD_EHIP, MAD_EOVERFLOW, MAD_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5
MAD_FP32, MAD_BF16, MAD_FP8_E4M3 = 0, 1, 2
MAD_FLAG_NONE, MAD_FLAG_NO_CHECK, MAD_FLAG_TIMING, MAD_FLAG_GRAM = 0, 1, 2, 4
MAD_FLAG_SQUARE = 8
MAD_OPT_ACCUM, MAD_OPT_SAMPLER_ORDER, MAD_OPT_ORDER_CHUNK = 0, 1, 2
MAD_ACCUM_PAIRS, MAD_ACCUM_HASH = 0, 1

# every symbol include/mad.h declares
EXPORTS = (
    "mad_plan_create_dense", "mad_plan_create_csr", "mad_plan_refresh",
    "mad_plan_topk", "mad_topk", "mad_plan_destroy", "mad_plan_stats",
    "mad_last_error", "mad_debug_table", "mad_debug_norms",
    "mad_debug_samples", "mad_debug_scores", "mad_debug_candidates",
    "mad_fix_exponent", "mad_plan_phase_ms", "mad_probe_memory",
    "mad_bruteforce_topk", "mips_plan_create", "mips_topk_batch",
    "mips_get_config", "mips_set_config", "mips_autotune", "mips_stats",
    "mips_debug_scores", "mad_plan_set_verify_precision",
    "mad_plan_verify_stats", "mad_debug_accumulate", "mad_plan_set_option",
    "mad_plan_get_option", "mad_accumulate_noalloc",
    "mad_bruteforce_topk_csr", "mad_debug_lowp_screen",
    "mips_get_table_factor", "mips_set_table_factor", "mips_autotune_cache",
)


class MadError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


_lib = None
_P, _i64, _u64, _i32, _u32 = (C.c_void_p, C.c_int64, C.c_uint64, C.c_int32,
                              C.c_uint32)


def lib():
    """Load libmad.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmad.so is not built: run "
                              "python -m paper_1506_03872_amd.build")
        L = C.CDLL(LIB_PATH)
        L.mad_last_error.restype = C.c_char_p
        L.mad_plan_create_dense.argtypes = [_P, _i64, _P, _i64, _i64, _u32,
                                            _P, C.POINTER(_P)]
        L.mad_plan_create_csr.argtypes = [_P, _P, _P, _i64, _P, _P, _P, _i64,
                                          _i64, _u32, _P, C.POINTER(_P)]
        L.mad_plan_refresh.argtypes = [_P, _P]
        L.mad_plan_topk.argtypes = [_P, _i64, _i64, _i64, _u64, _P, _P, _P]
        L.mad_topk.argtypes = [_P, _i64, _P, _i64, _i64, _i64, _i64, _i64,
                               _u64, _P, _P, _P]
        L.mad_plan_destroy.argtypes = [_P]
        L.mad_plan_destroy.restype = None
        L.mad_plan_stats.argtypes = [_P, _P, _P, _P, _P, _P]
        L.mad_debug_table.argtypes = [_P, C.c_int, _i64, _P, _P, _P, _i64, _P]
        L.mad_debug_norms.argtypes = [_P, _P, _P, _P, _P]
        L.mad_debug_samples.argtypes = [_P, _u64, _u64, _i64, _i64, C.c_int,
                                        _P, _P, _P, _P, _P, _P]
        L.mad_debug_scores.argtypes = [_P, _P, _P, _i64, _P, _P]
        L.mad_debug_accumulate.argtypes = [_P, _P, _i64, C.c_int, _P, _P,
                                           _i64, _P, _P]
        L.mad_debug_candidates.argtypes = [_P, _P, _P, _P, _i64, _P]
        L.mad_fix_exponent.argtypes = [_P, _i64, _P]
        L.mad_plan_phase_ms.argtypes = [_P, _P, C.c_int]
        L.mad_probe_memory.argtypes = [C.c_int, _P, _i64, _i64, _u64, _P]
        L.mad_bruteforce_topk.argtypes = [_P, _i64, _P, _i64, _i64, C.c_int,
                                          _i64, _i64, _P, _P, _P, _P]
        L.mad_plan_set_verify_precision.argtypes = [_P, C.c_int, _P]
        L.mad_plan_verify_stats.argtypes = [_P, _P, _P]
        L.mad_accumulate_noalloc.argtypes = [_P, _P, _i64, C.c_int, _P, _P,
                                             _P, _P]
        L.mad_bruteforce_topk_csr.argtypes = [_P, _P, _P, _i64, _P, _P, _P,
                                              _i64, _i64, C.c_int, _i64,
                                              _i64, _P, _P, _P, _P]
        L.mad_debug_lowp_screen.argtypes = [_P, _P, _i64, _P, _P, _P]
        L.mad_plan_set_option.argtypes = [_P, C.c_int, _i64]
        L.mad_plan_get_option.argtypes = [_P, C.c_int, _P]
        L.mips_plan_create.argtypes = [_P, _i64, _i64, _u32, _P,
                                       C.POINTER(_P)]
        L.mips_topk_batch.argtypes = [_P, _P, _i64, _P, _P, _i64, _u64, _P,
                                      _P, _P]
        L.mips_get_config.argtypes = [_P, _P, _P, _P]
        L.mips_set_config.argtypes = [_P, C.c_int, C.c_int, C.c_int]
        L.mips_autotune.argtypes = [_P, _P, _i64, _P, _P, _i64, _u64, _P, _P,
                                    C.c_int, _P, _P]
        L.mips_get_table_factor.argtypes = [_P, _P]
        L.mips_set_table_factor.argtypes = [_P, C.c_int]
        L.mips_autotune_cache.argtypes = [_P, C.c_char_p]
        L.mips_stats.argtypes = [_P, _P, _P, _P, _P]
        L.mips_debug_scores.argtypes = [_P, _i64, _P, _P, _i64, _P, _P]
        _lib = L
    return _lib


def _check(rc):
    if rc != MAD_OK:
        raise MadError(rc, lib().mad_last_error().decode())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be contiguous %s" % (name, dtype))
    return C.c_void_p(t.data_ptr())


def _dev_opt(t, dtype, name):
    """_dev, allowing an empty tensor (null data pointer)."""
    if t.numel() == 0:
        return C.c_void_p(0)
    return _dev(t, dtype, name)


def unpack_pairs(raw, n):
    """mad_pair records (a (t, 3) int64 tensor) -> dict of i, j, c, x."""
    import torch
    r = raw[:n]
    if n == 0:
        e = torch.empty(0, dtype=torch.int64, device=raw.device)
        f = torch.empty(0, dtype=torch.float32, device=raw.device)
        return dict(i=e, j=e.clone(), c=f, x=f.clone())
    cx = r[:, 2].clone(memory_format=torch.contiguous_format)
    cx = cx.view(torch.float32).view(-1, 2)
    return dict(i=r[:, 0].clone(), j=r[:, 1].clone(), c=cx[:, 0].clone(),
                x=cx[:, 1].clone())


class Plan:
    """Owning handle of a mad_plan (tables of Alg. 3 for one A, B)."""

    def __init__(self, handle, keep, m, n, d):
        self._h = handle
        self._keep = keep
        self.m, self.n, self.d = m, n, d

    @classmethod
    def dense(cls, A, B, flags=MAD_FLAG_NONE, stream=None):
        import torch
        m, d = A.shape
        n, d2 = B.shape
        if d != d2:
            raise ValueError("A and B must have the same dimension")
        h = C.c_void_p()
        _check(lib().mad_plan_create_dense(
            _dev(A, torch.float32, "A"), m, _dev(B, torch.float32, "B"), n, d,
            flags, _stream(stream), C.byref(h)))
        return cls(h, (A, B), m, n, d)

    @classmethod
    def csr(cls, a, b, m, n, d, flags=MAD_FLAG_NONE, stream=None):
        """Sparse plan: a = (ptr int64 m+1, idx int32, val fp32) CUDA tensors
        of A's compressed rows, b likewise for B."""
        import torch
        (ap, ai, av), (bp, bi, bv) = a, b
        h = C.c_void_p()
        _check(lib().mad_plan_create_csr(
            _dev(ap, torch.int64, "a_ptr"), _dev_opt(ai, torch.int32, "a_idx"),
            _dev_opt(av, torch.float32, "a_val"), m,
            _dev(bp, torch.int64, "b_ptr"), _dev_opt(bi, torch.int32, "b_idx"),
            _dev_opt(bv, torch.float32, "b_val"), n, d, flags,
            _stream(stream), C.byref(h)))
        return cls(h, (a, b), m, n, d)

    def refresh(self, stream=None):
        _check(lib().mad_plan_refresh(self._h, _stream(stream)))

    def close(self):
        if self._h:
            lib().mad_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def topk_raw(self, t, s, t_prime, seed, out, n_out, stream=None):
        """Enqueue mad_plan_topk into caller-owned out ((t,3) int64) and
        n_out ((1,) int64) without synchronising."""
        import torch
        _check(lib().mad_plan_topk(self._h, t, s, t_prime, seed,
                                   _dev(out, torch.int64, "out"),
                                   _dev(n_out, torch.int64, "n_out"),
                                   _stream(stream)))

    def topk(self, t, s, t_prime, seed=0, stream=None):
        import torch
        out = torch.empty((t, 3), dtype=torch.int64, device="cuda")
        n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.topk_raw(t, s, t_prime, seed, out, n_out, stream)
        torch.cuda.synchronize()
        return unpack_pairs(out, int(n_out.item()))

    def stats(self):
        w = C.c_double()
        cl, di, npos, nc = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().mad_plan_stats(self._h, C.byref(w), C.byref(cl),
                                    C.byref(di), C.byref(npos), C.byref(nc)))
        return dict(wnorm=w.value, closed=cl.value, distinct=di.value,
                    n_pos=npos.value, n_cand=nc.value)

    def set_verify_precision(self, precision, stream=None):
        _check(lib().mad_plan_set_verify_precision(self._h, precision,
                                                   _stream(stream)))

    def set_option(self, option, value):
        """mad_plan_set_option: a launch choice (MAD_OPT_*), result-invariant."""
        _check(lib().mad_plan_set_option(self._h, option, value))

    def get_option(self, option):
        v = C.c_int64()
        _check(lib().mad_plan_get_option(self._h, option, C.byref(v)))
        return v.value

    def verify_stats(self):
        nc, nr = C.c_int64(), C.c_int64()
        _check(lib().mad_plan_verify_stats(self._h, C.byref(nc), C.byref(nr)))
        return dict(n_cand=nc.value, n_reranked=nr.value)

    def phase_ms(self):
        """[tables, sampling, postprocess, clear, accumulate, sampling
        kernel] ms of the last calls (needs MAD_FLAG_TIMING)."""
        arr = (C.c_double * 6)()
        _check(lib().mad_plan_phase_ms(self._h, arr, 6))
        return list(arr)

    def fix_exponent(self, s):
        F = C.c_int()
        _check(lib().mad_fix_exponent(self._h, s, C.byref(F)))
        return F.value

    # ---- parity / debug ----------------------------------------------------
    def table(self, which, idx=0):
        import numpy as np
        ns = C.c_int64()
        _check(lib().mad_debug_table(self._h, which, idx, None, None, None, 0,
                                     C.byref(ns)))
        thr = np.zeros(ns.value, np.uint32)
        al = np.zeros(ns.value, np.uint32)
        item = np.zeros(ns.value, np.int32)
        _check(lib().mad_debug_table(
            self._h, which, idx, thr.ctypes.data_as(_P), al.ctypes.data_as(_P),
            item.ctypes.data_as(_P), ns.value, C.byref(ns)))
        return thr, al, item

    def norms(self):
        import numpy as np
        na = np.zeros(self.m, np.float64)
        nb = np.zeros(self.d, np.float64)
        v = np.zeros(self.d, np.float64)
        om = np.zeros(self.d, np.float64)
        _check(lib().mad_debug_norms(self._h, na.ctypes.data_as(_P),
                                     nb.ctypes.data_as(_P),
                                     v.ctypes.data_as(_P),
                                     om.ctypes.data_as(_P)))
        return na, nb, v, om

    def samples(self, seed, l0, count, F, qid=0, stream=None):
        import torch
        dev = "cuda"
        k = torch.empty(count, dtype=torch.int32, device=dev)
        i = torch.empty(count, dtype=torch.int32, device=dev)
        j = torch.empty(count, dtype=torch.int32, device=dev)
        kp = torch.empty(count, dtype=torch.int32, device=dev)
        inc = torch.empty(count, dtype=torch.int64, device=dev)
        _check(lib().mad_debug_samples(
            self._h, seed, qid, l0, count, F, C.c_void_p(k.data_ptr()),
            C.c_void_p(i.data_ptr()), C.c_void_p(j.data_ptr()),
            C.c_void_p(kp.data_ptr()), C.c_void_p(inc.data_ptr()),
            _stream(stream)))
        return dict(k=k.cpu().numpy(), i=i.cpu().numpy(), j=j.cpu().numpy(),
                    kp=kp.cpu().numpy(), inc=inc.cpu().numpy())

    def scores(self):
        """X of the last topk: (keys, x_fix) sorted by key, and F."""
        import numpy as np
        import torch
        n = C.c_int64()
        F = C.c_int()
        _check(lib().mad_debug_scores(self._h, None, None, 0, C.byref(n),
                                      C.byref(F)))
        cap = max(n.value, 1)
        keys = torch.empty(cap, dtype=torch.int64, device="cuda")
        x = torch.empty(cap, dtype=torch.int64, device="cuda")
        _check(lib().mad_debug_scores(self._h, C.c_void_p(keys.data_ptr()),
                                      C.c_void_p(x.data_ptr()), cap,
                                      C.byref(n), C.byref(F)))
        keys = keys[:n.value].cpu().numpy()
        x = x[:n.value].cpu().numpy()
        o = np.argsort(keys, kind="stable")
        return keys[o], x[o], F.value

    def lowp_screen(self, keys, stream=None):
        """(c^, margin) of the low-precision screen for CUDA int64 keys
        i*n + j (plan with bf16 / fp8 verification), as numpy arrays."""
        import torch
        n = int(keys.numel())
        ch = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        mg = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        _check(lib().mad_debug_lowp_screen(
            self._h, _dev_opt(keys, torch.int64, "keys"), n,
            C.c_void_p(ch.data_ptr()), C.c_void_p(mg.data_ptr()),
            _stream(stream)))
        torch.cuda.synchronize()
        return ch[:n].cpu().numpy(), mg[:n].cpu().numpy()

    def candidates(self):
        """Omega_t' of the last topk, sorted by key: keys, x_fix, c."""
        import numpy as np
        import torch
        n = C.c_int64()
        _check(lib().mad_debug_candidates(self._h, None, None, None, 0,
                                          C.byref(n)))
        cap = max(n.value, 1)
        keys = torch.empty(cap, dtype=torch.int64, device="cuda")
        x = torch.empty(cap, dtype=torch.int64, device="cuda")
        c = torch.empty(cap, dtype=torch.float32, device="cuda")
        _check(lib().mad_debug_candidates(
            self._h, C.c_void_p(keys.data_ptr()), C.c_void_p(x.data_ptr()),
            C.c_void_p(c.data_ptr()), cap, C.byref(n)))
        keys = keys[:n.value].cpu().numpy()
        o = np.argsort(keys, kind="stable")
        return keys[o], x[:n.value].cpu().numpy()[o], c[:n.value].cpu().numpy()[o]


class MipsPlan(Plan):
    """Owning handle of a MIPS plan: the database tables (A side of Alg. 3)
    shared by batches of queries."""

    @classmethod
    def create(cls, A, flags=MAD_FLAG_NONE, stream=None):
        import torch
        m, d = A.shape
        h = C.c_void_p()
        _check(lib().mips_plan_create(_dev(A, torch.float32, "A"), m, d,
                                      flags, _stream(stream), C.byref(h)))
        return cls(h, (A,), m, 1, d)

    @staticmethod
    def _budgets(s, tp):
        import numpy as np
        s = np.ascontiguousarray(s, dtype=np.int64)
        tp = np.ascontiguousarray(tp, dtype=np.int64)
        return s, tp

    def batch_raw(self, Q, s, tp, t, seed, out, n_out, stream=None):
        """Enqueue mips_topk_batch: Q (nq, d) fp32, s / tp host int64
        arrays, out (nq*t, 3) int64, n_out (nq,) int64."""
        import torch
        s, tp = self._budgets(s, tp)
        nq = Q.shape[0]
        self._keep_q = (Q, s, tp, out, n_out)
        _check(lib().mips_topk_batch(
            self._h, _dev(Q, torch.float32, "Q"), nq, s.ctypes.data_as(_P),
            tp.ctypes.data_as(_P), t, seed, _dev(out, torch.int64, "out"),
            _dev(n_out, torch.int64, "n_out"), _stream(stream)))

    def batch(self, Q, s, tp, t, seed=0, stream=None):
        """Synchronous batch: list of dicts (i, j, c, x) per query; a query
        with non-finite values gives None."""
        import torch
        nq = Q.shape[0]
        out = torch.empty((max(nq, 1) * t, 3), dtype=torch.int64,
                          device="cuda")
        n_out = torch.zeros(max(nq, 1), dtype=torch.int64, device="cuda")
        self.batch_raw(Q, s, tp, t, seed, out, n_out, stream)
        torch.cuda.synchronize()
        cnt = n_out.cpu().tolist()
        res = []
        for q in range(nq):
            if cnt[q] < 0:
                res.append(None)
            else:
                res.append(unpack_pairs(out[q * t:(q + 1) * t], cnt[q]))
        return res

    def config(self):
        c, u, g = C.c_int(), C.c_int(), C.c_int()
        _check(lib().mips_get_config(self._h, C.byref(c), C.byref(u),
                                     C.byref(g)))
        return dict(chunk=c.value, unroll=u.value, grid=g.value)

    def set_config(self, chunk, unroll, grid):
        _check(lib().mips_set_config(self._h, chunk, unroll, grid))

    def table_factor(self):
        f = C.c_int()
        _check(lib().mips_get_table_factor(self._h, C.byref(f)))
        return f.value

    def set_table_factor(self, slots_per_key):
        _check(lib().mips_set_table_factor(self._h, slots_per_key))

    def set_autotune_cache(self, path):
        """File of the autotuner's choices (None: none)."""
        _check(lib().mips_autotune_cache(
            self._h, None if path is None else str(path).encode()))

    def autotune(self, Q, s, tp, t, seed=0, reps=2, stream=None):
        import torch
        s, tp = self._budgets(s, tp)
        nq = Q.shape[0]
        out = torch.empty((max(nq, 1) * t, 3), dtype=torch.int64,
                          device="cuda")
        n_out = torch.zeros(max(nq, 1), dtype=torch.int64, device="cuda")
        best = C.c_double()
        _check(lib().mips_autotune(
            self._h, _dev(Q, torch.float32, "Q"), nq, s.ctypes.data_as(_P),
            tp.ctypes.data_as(_P), t, seed, _dev(out, torch.int64, "out"),
            _dev(n_out, torch.int64, "n_out"), reps, _stream(stream),
            C.byref(best)))
        return dict(self.config(), slots=self.table_factor(), ms=best.value)

    def mips_stats(self, nq):
        import numpy as np
        npos = np.zeros(max(nq, 1), np.int64)
        ncand = np.zeros(max(nq, 1), np.int64)
        cl, di = C.c_int64(), C.c_int64()
        _check(lib().mips_stats(self._h, npos.ctypes.data_as(_P),
                                ncand.ctypes.data_as(_P), C.byref(cl),
                                C.byref(di)))
        return dict(n_pos=npos[:nq], n_cand=ncand[:nq], closed=cl.value,
                    distinct=di.value)

    def query_scores(self, q):
        """Score table of query q after the last batch: (keys i, x_fix)
        sorted by key, and F."""
        import numpy as np
        import torch
        n = C.c_int64()
        F = C.c_int()
        _check(lib().mips_debug_scores(self._h, q, None, None, 0, C.byref(n),
                                       C.byref(F)))
        cap = max(n.value, 1)
        keys = torch.empty(cap, dtype=torch.int64, device="cuda")
        x = torch.empty(cap, dtype=torch.int64, device="cuda")
        _check(lib().mips_debug_scores(self._h, q, C.c_void_p(keys.data_ptr()),
                                       C.c_void_p(x.data_ptr()), cap,
                                       C.byref(n), C.byref(F)))
        keys = keys[:n.value].cpu().numpy()
        x = x[:n.value].cpu().numpy()
        o = np.argsort(keys, kind="stable")
        return keys[o], x[o], F.value


class BfStats(C.Structure):
    _fields_ = [("ms_screen", C.c_double), ("ms_filter", C.c_double),
                ("ms_rerank", C.c_double), ("candidates", C.c_int64),
                ("tau", C.c_float), ("row_stride", C.c_int64),
                ("reranked", C.c_int64)]


def bruteforce_topk(A, B, t, precision=MAD_FP32, t_screen=0, stream=None):
    """Exhaustive top-t by |a_i . b_j| on the matrix cores (synchronises).
    Returns (dict of i, j, c, x, stats dict)."""
    import torch
    m, d = A.shape
    n = B.shape[0]
    out = torch.empty((t, 3), dtype=torch.int64, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = BfStats()
    _check(lib().mad_bruteforce_topk(
        _dev(A, torch.float32, "A"), m, _dev(B, torch.float32, "B"), n, d,
        precision, t, t_screen, C.c_void_p(out.data_ptr()),
        C.c_void_p(n_out.data_ptr()), C.byref(st), _stream(stream)))
    stats = {f: getattr(st, f) for f, _ in BfStats._fields_}
    return unpack_pairs(out, int(n_out.item())), stats


class BfCsrStats(C.Structure):
    _fields_ = [("ms_split", C.c_double), ("ms_heavy", C.c_double),
                ("ms_light", C.c_double), ("ms_final", C.c_double),
                ("heavy", C.c_int64), ("wedges", C.c_int64),
                ("light_wedges", C.c_int64),
                ("heavy_candidates", C.c_int64),
                ("light_candidates", C.c_int64), ("candidates", C.c_int64),
                ("tau", C.c_float)]


def bruteforce_topk_csr(a, b, m, n, d, t, precision=MAD_FP32, heavy=0,
                        stream=None):
    """Exhaustive top-t by |a_i . b_j| of sparse inputs (synchronises): a, b
    are (ptr int64, idx int32, val fp32) CUDA tensors of the compressed
    rows.  Returns (dict of i, j, c, x, stats dict)."""
    import torch
    (ap, ai, av), (bp, bi, bv) = a, b
    out = torch.empty((t, 3), dtype=torch.int64, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = BfCsrStats()
    _check(lib().mad_bruteforce_topk_csr(
        _dev(ap, torch.int64, "a_ptr"), _dev_opt(ai, torch.int32, "a_idx"),
        _dev_opt(av, torch.float32, "a_val"), m,
        _dev(bp, torch.int64, "b_ptr"), _dev_opt(bi, torch.int32, "b_idx"),
        _dev_opt(bv, torch.float32, "b_val"), n, d, precision, t, heavy,
        C.c_void_p(out.data_ptr()), C.c_void_p(n_out.data_ptr()),
        C.byref(st), _stream(stream)))
    stats = {f: getattr(st, f) for f, _ in BfCsrStats._fields_}
    return unpack_pairs(out, int(n_out.item())), stats


def debug_accumulate(keys, vals, F):
    """The score accumulation alone: keys (CUDA uint64 as int64, -1 = none)
    and vals (CUDA float32) -> (distinct keys, int64 sums of rne(v 2^F))
    as numpy arrays sorted by key."""
    import numpy as np
    import torch
    n = int(keys.numel())
    assert vals.numel() == n
    kp = _dev(keys, torch.int64, "keys") if n else None
    vp = _dev(vals, torch.float32, "vals") if n else None
    got = C.c_int64()
    cap = max(n, 1)
    ok = torch.empty(cap, dtype=torch.int64, device="cuda")
    ox = torch.empty(cap, dtype=torch.int64, device="cuda")
    _check(lib().mad_debug_accumulate(kp, vp, n, F,
                                      C.c_void_p(ok.data_ptr()),
                                      C.c_void_p(ox.data_ptr()), cap,
                                      C.byref(got), None))
    k = ok[:got.value].cpu().numpy()
    x = ox[:got.value].cpu().numpy()
    o = np.argsort(k, kind="stable")
    return k[o], x[o]


def accumulate_noalloc(keys, vals, F, out_keys, out_x, n_out, stream=None):
    """mad_accumulate_noalloc: the score accumulation in the library's static
    workspace (no device allocation, no synchronisation).  keys (CUDA int64,
    -1 = none) and vals (CUDA float32) of n <= 2^18 pairs; out_keys, out_x
    (CUDA int64, capacity n) and n_out (CUDA int64, one entry) receive the
    distinct keys, their sums and their count."""
    import torch
    n = int(keys.numel())
    kp = _dev(keys, torch.int64, "keys") if n else None
    vp = _dev(vals, torch.float32, "vals") if n else None
    okp = _dev(out_keys, torch.int64, "out_keys") if n else None
    oxp = _dev(out_x, torch.int64, "out_x") if n else None
    _check(lib().mad_accumulate_noalloc(kp, vp, n, F, okp, oxp,
                                        _dev(n_out, torch.int64, "n_out"),
                                        _stream(stream)))


def probe_memory(kind, buf, nops, seed=0, stream=None):
    """Enqueue one mad_probe_memory run over buf (a CUDA int64 tensor whose
    length is a power of two)."""
    import torch
    _check(lib().mad_probe_memory(kind, _dev(buf, torch.int64, "buf"),
                                  buf.numel(), nops, seed, _stream(stream)))


def topk(A, B, t, s, t_prime, seed=0, stream=None):
    """One-shot mad_topk: returns dict(i, j, c, x) (synchronises)."""
    import torch
    m, d = A.shape
    n = B.shape[0]
    out = torch.empty((t, 3), dtype=torch.int64, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    _check(lib().mad_topk(_dev(A, torch.float32, "A"), m,
                          _dev(B, torch.float32, "B"), n, d, t, s, t_prime,
                          seed, C.c_void_p(out.data_ptr()),
                          C.c_void_p(n_out.data_ptr()), _stream(stream)))
    return unpack_pairs(out, int(n_out.item()))

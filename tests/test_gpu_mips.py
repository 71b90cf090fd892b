"""GPU parity of the MIPS batch: every query of a batch against the oracle's
general plan with B = {q} (n = 1) and Philox counter word 1 = q.

Bar: the database tables and each query's score table X are bit-exact, the
per-query candidate counts are equal, and each query's top t matches the
oracle's (indices exact up to swaps within the fp32 tolerance at the t-th
value; c within 1e-5 of sum_k |a_ik q_k|)."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5
SEED = 31


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


def _db(m=3000, d=40, nq=8, seed=0):
    A, Q, _ = workloads.mips(m, d, nq, seed=seed)
    Q[5] = 0.0  # a zero query: ||W||_1 = 0, no samples can be drawn
    return A, Q


S = np.array([0, 50, 300, 5000, 20000, 1500, 700, 9000], np.int64)
TP = np.array([10, 10, 20, 100, 10**6, 50, 5, 40], np.int64)
T = 5


def _check_query(A, q, qvec, g, o, t):
    """g: GPU result dict of query q; o: the oracle's topk dict."""
    gi = g["i"].cpu().numpy()
    assert np.all(g["j"].cpu().numpy() == q)
    gc = g["c"].cpu().numpy().astype(np.float64)
    assert len(gi) == len(o["key"])
    c64 = (A[gi].astype(np.float64) * qvec.astype(np.float64)).sum(1)
    scale = (np.abs(A[gi].astype(np.float64)) *
             np.abs(qvec.astype(np.float64))).sum(1)
    assert np.all(np.abs(gc - c64) <= TOL * scale + 1e-30)
    if np.array_equal(gi, o["key"]):
        gx = g["x"].cpu().numpy().astype(np.float64)
        ox = np.ldexp(o["x"].astype(np.float64), -o["F"]).astype(np.float32)
        assert np.array_equal(gx.astype(np.float32), ox)
        return
    ok = set(o["key"].tolist())
    tau = np.abs(o["c"]).min() if len(o["c"]) else 0.0
    for i, c, sc in zip(gi.tolist(), c64.tolist(), scale.tolist()):
        if i not in ok:
            assert abs(abs(c) - tau) <= 2 * TOL * sc, (q, i)


def _oracle_query(A, qvec, q, s, tp, t, seed=SEED):
    # a batch keeps each score beside its key i + 1 in one 64-bit slot, so
    # its exponent is taken with the key's bits (the bit length of m)
    op = oracle.Plan.dense(A, qvec[None, :].copy())
    F = op.fix_exponent(int(s), key_bits=int(A.shape[0]).bit_length())
    o = op.topk(seed=seed, s=int(s), t_prime=int(tp), t=t, F=F, qid=q)
    keys, x, closed = op.scores(seed=seed, s=int(s), F=o["F"], qid=q)
    op.close()
    return o, keys, x, closed


def test_database_tables_bitexact(mad_gpu):
    A, Q = _db()
    gp = mad_gpu.MipsPlan.create(to_dev(A))
    op = oracle.Plan.dense(A, Q[:1].copy())
    gna, _, gv, _ = _mips_norms(gp)
    ona, _, ov, _ = op.norms()
    assert np.array_equal(gna, ona) and np.array_equal(gv, ov)
    m, d = A.shape
    for which, idx in [(1, 0), (1, d // 2), (1, d - 1), (3, 0), (3, m // 3),
                       (3, m - 1)]:
        gthr, gal, _ = gp.table(which, idx)
        othr, oal, _, _, _, _ = op.table(which, idx)
        assert np.array_equal(gthr, othr) and np.array_equal(gal, oal)
    gp.close()
    op.close()


def _mips_norms(gp):
    import ctypes as C
    import paper_1506_03872_amd as mad
    na = np.zeros(gp.m, np.float64)
    v = np.zeros(gp.d, np.float64)
    mad._check(mad.lib().mad_debug_norms(gp._h, na.ctypes.data_as(C.c_void_p),
                                         None, v.ctypes.data_as(C.c_void_p),
                                         None))
    return na, None, v, None


def test_batch_matches_oracle_per_query(mad_gpu):
    A, Q = _db()
    gp = mad_gpu.MipsPlan.create(to_dev(A))
    Qd = to_dev(Q)
    say("batch nq=%d budgets=%s" % (len(S), S.tolist()))
    res = gp.batch(Qd, S, TP, T, seed=SEED)
    st = gp.mips_stats(len(S))
    tot_closed = 0
    for q in range(len(S)):
        say("query", q, "s", int(S[q]))
        if S[q] == 0 or q == 5:
            assert res[q] is not None and len(res[q]["i"]) == 0
            assert st["n_pos"][q] == 0
            continue
        o, ok, ox, closed = _oracle_query(A, Q[q], q, S[q], TP[q], T)
        tot_closed += closed
        gk, gx, F = gp.query_scores(q)
        assert F == o["F"]
        assert np.array_equal(gk, ok) and np.array_equal(gx, ox)
        assert st["n_pos"][q] == o["n_pos"]
        assert st["n_cand"][q] == len(o["tp_key"])
        _check_query(A, q, Q[q], res[q], o, T)
    assert st["closed"] == tot_closed
    gp.close()


def test_graph_replay_and_shapes_do_not_change_results(mad_gpu):
    import torch
    A, Q = _db(m=2000, d=24, nq=8, seed=1)
    gp = mad_gpu.MipsPlan.create(to_dev(A))
    Qd = to_dev(Q)
    nq = len(S)
    out = torch.empty((nq * T, 3), dtype=torch.int64, device="cuda")
    n_out = torch.zeros(nq, dtype=torch.int64, device="cuda")
    gp.batch_raw(Qd, S, TP, T, SEED, out, n_out)
    torch.cuda.synchronize()
    ref = (out.clone(), n_out.clone())
    for rep in range(3):  # graph replays with eager work in between
        out.fill_(-7)
        n_out.fill_(-7)
        gp.batch_raw(Qd, S, TP, T, SEED, out, n_out)
        torch.cuda.synchronize()
        assert torch.equal(n_out, ref[1]), rep
        for q in range(nq):
            k = int(ref[1][q])
            assert torch.equal(out[q * T:q * T + k], ref[0][q * T:q * T + k])
    for chunk, unroll, grid in ((256, 1, 7), (65536, 8, 4096), (1024, 2, 300)):
        gp.set_config(chunk, unroll, grid)
        r = gp.batch(Qd, S, TP, T, seed=SEED)
        for q in range(nq):
            k = int(ref[1][q])
            assert np.array_equal(r[q]["i"].cpu().numpy(),
                                  ref[0][q * T:q * T + k, 0].cpu().numpy())
    # a new seed re-captures and still agrees with the oracle
    r = gp.batch(Qd, S, TP, T, seed=SEED + 1)
    o, _, _, _ = _oracle_query(A, Q[4], 4, S[4], TP[4], T, seed=SEED + 1)
    _check_query(A, 4, Q[4], r[4], o, T)
    gp.close()


def test_autotune_keeps_results(mad_gpu):
    A, Q = _db(m=1500, d=16, nq=8, seed=2)
    gp = mad_gpu.MipsPlan.create(to_dev(A))
    Qd = to_dev(Q)
    before = gp.batch(Qd, S, TP, T, seed=SEED)
    tuned = gp.autotune(Qd, S, TP, T, seed=SEED, reps=1)
    say("tuned", tuned)
    assert tuned["ms"] > 0
    after = gp.batch(Qd, S, TP, T, seed=SEED)
    for q in range(len(S)):
        assert np.array_equal(before[q]["i"].cpu().numpy(),
                              after[q]["i"].cpu().numpy())
        assert np.array_equal(before[q]["c"].cpu().numpy(),
                              after[q]["c"].cpu().numpy())
    gp.close()


def test_timing_mode_and_nonfinite_query(mad_gpu):
    A, Q = _db(m=1200, d=32, nq=8, seed=3)
    Q[2, 7] = np.nan
    gp = mad_gpu.MipsPlan.create(to_dev(A), flags=mad_gpu.MAD_FLAG_TIMING)
    res = gp.batch(to_dev(Q), S, TP, T, seed=SEED)
    assert res[2] is None
    ph = gp.phase_ms()
    # query tables, sampling, postprocessing, graph set-up; no pair
    # accumulation phase in a batch
    assert all(v >= 0 for v in ph[:4]) and ph[4] == -1.0
    o, _, _, _ = _oracle_query(A, Q[3], 3, S[3], TP[3], T)
    _check_query(A, 3, Q[3], res[3], o, T)
    gp.close()


def test_invalid_arguments(mad_gpu):
    A, Q = _db(m=500, d=8, nq=8, seed=4)
    gp = mad_gpu.MipsPlan.create(to_dev(A))
    Qd = to_dev(Q)
    with pytest.raises(mad_gpu.MadError):
        gp.batch(Qd, S, TP, 1025)
    with pytest.raises(mad_gpu.MadError):
        gp.batch(Qd, S, np.full(len(S), 2), 5)  # t' < t
    with pytest.raises(mad_gpu.MadError):
        gp.batch(Qd, -S - 1, TP, 5)
    with pytest.raises(mad_gpu.MadError):  # a MIPS plan is not a MAD plan
        gp.topk(t=5, s=10, t_prime=10)
    empty = gp.batch(Qd[:0], S[:0], TP[:0], 5)
    assert empty == []
    gp.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_low_precision_screen_keeps_results(mad_gpu, prec):
    # bf16 / fp8 screening of each query's candidates before the fp32
    # verification: the top t (indices, c, x) must be exactly the fp32 one,
    # in graph replays and eagerly, and bf16 must skip most fp32 rows
    A, Q = _db(m=4000, d=64, nq=8, seed=4)
    Qd = to_dev(Q)
    for flags in (0, mad_gpu.MAD_FLAG_TIMING):
        gp = mad_gpu.MipsPlan.create(to_dev(A), flags=flags)
        ref = gp.batch(Qd, S, TP, T, seed=SEED)
        st0 = gp.verify_stats()
        assert st0["n_reranked"] == st0["n_cand"]
        gp.set_verify_precision(prec)
        for rep in range(2):
            got = gp.batch(Qd, S, TP, T, seed=SEED)
            for q in range(len(S)):
                if ref[q] is None:
                    assert got[q] is None
                    continue
                for key in ("i", "c", "x"):
                    assert np.array_equal(got[q][key].cpu().numpy(),
                                          ref[q][key].cpu().numpy()), (q, key)
            if rep == 0 and flags == 0:  # against the oracle, query by query
                for q in range(len(S)):
                    if got[q] is None or q == 5 or S[q] == 0:
                        continue
                    o, _, _, _ = _oracle_query(A, Q[q], q, S[q], TP[q], T)
                    _check_query(A, q, Q[q], got[q], o, T)
        st = gp.verify_stats()
        say("flags", flags, "prec", prec, st0, st)
        assert st["n_cand"] == st0["n_cand"]
        assert st["n_reranked"] <= st["n_cand"]
        if prec == 1:
            assert st["n_reranked"] < st["n_cand"] // 4
        gp.set_verify_precision(mad_gpu.MAD_FP32)
        back = gp.batch(Qd, S, TP, T, seed=SEED)
        for q in range(len(S)):
            if ref[q] is not None:
                assert np.array_equal(back[q]["i"].cpu().numpy(),
                                      ref[q]["i"].cpu().numpy())
        gp.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_tied_scores_take_the_digit_selection(mad_gpu, prec):
    # Every database row is +v or -v, so every candidate has the same |c|
    # and the final top t is decided by i alone, among more candidates than
    # the post kernel's LDS list holds (2048); with the bf16 screen, every
    # candidate also survives it.  Both take the general selection paths.
    m, d = 5000, 16
    V, Qg = workloads.dense_gaussian(1, 2, d, seed=7)
    sgn = np.where((np.arange(m) * 2654435761) % 7 < 3, -1.0, 1.0)
    A = (sgn[:, None] * V[0][None, :]).astype(np.float32)
    s = np.array([40000, 30000], np.int64)
    tp = np.array([10**6, 10**6], np.int64)
    gp = mad_gpu.MipsPlan.create(to_dev(A))
    if prec:
        gp.set_verify_precision(prec)
    res = gp.batch(to_dev(Qg), s, tp, T, seed=SEED)
    st = gp.mips_stats(2)
    for q in range(2):
        say("query", q, "candidates", int(st["n_cand"][q]))
        assert st["n_cand"][q] > 2048
        o, _, _, _ = _oracle_query(A, Qg[q], q, s[q], tp[q], T)
        assert np.array_equal(res[q]["i"].cpu().numpy(), o["key"])
        _check_query(A, q, Qg[q], res[q], o, T)
    gp.close()


def test_table_factor_and_choice_file(mad_gpu, tmp_path):
    # The score tables' slots per key never change a result.  With a
    # choice file, a second plan takes the first plan's tuned choice for
    # the same batch without trials, and the file keeps one line.
    A, Q = _db(m=2000, d=32, nq=8, seed=6)
    Qd = to_dev(Q)
    gp = mad_gpu.MipsPlan.create(to_dev(A))
    ref = gp.batch(Qd, S, TP, T, seed=SEED)
    ref_x = {q: gp.query_scores(q) for q in (3, 4)}
    for f in (4, 8, 2):
        gp.set_table_factor(f)
        assert gp.table_factor() == f
        got = gp.batch(Qd, S, TP, T, seed=SEED)
        for q in range(len(S)):
            if ref[q] is None:
                assert got[q] is None
                continue
            for key in ("i", "c", "x"):
                assert np.array_equal(got[q][key].cpu().numpy(),
                                      ref[q][key].cpu().numpy()), (f, q, key)
        for q in (3, 4):
            k, x, F = gp.query_scores(q)
            assert np.array_equal(k, ref_x[q][0])
            assert np.array_equal(x, ref_x[q][1]) and F == ref_x[q][2]
    with pytest.raises(mad_gpu.MadError):
        gp.set_table_factor(3)
    path = tmp_path / "mips_choices.txt"
    gp.set_autotune_cache(path)
    first = gp.autotune(Qd, S, TP, T, seed=SEED, reps=1)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and " | " in lines[0]
    say("tuned", first, lines[0])
    gp2 = mad_gpu.MipsPlan.create(to_dev(A))
    gp2.set_autotune_cache(path)
    second = gp2.autotune(Qd, S, TP, T, seed=SEED, reps=1)
    for key in ("chunk", "unroll", "grid", "slots"):
        assert second[key] == first[key], key
    assert abs(second["ms"] - first["ms"]) < 1e-3
    assert len(path.read_text().splitlines()) == 1
    got = gp2.batch(Qd, S, TP, T, seed=SEED)
    for q in range(len(S)):
        if ref[q] is not None:
            assert np.array_equal(got[q]["i"].cpu().numpy(),
                                  ref[q]["i"].cpu().numpy())
    # another batch (other budgets) is tuned and appended
    gp2.autotune(Qd, S + 1, TP + 1, T, seed=SEED, reps=1)
    assert len(path.read_text().splitlines()) == 2
    gp.close()
    gp2.close()


@pytest.mark.parametrize("m", [4095, 4096])
def test_score_slot_key_width_at_its_boundary(mad_gpu, m):
    # The key field of a score slot has kb = bit length of m bits and holds
    # i + 1: m = 4095 fills a 12-bit field (i + 1 up to 4095 = 2^12 - 1),
    # m = 4096 takes 13 bits.  The rows near the end of the database carry
    # the largest keys; they are scaled up so that they are sampled.
    A, Q, _ = workloads.mips(m, 16, 2, seed=8)
    A[-8:] *= 6.0
    s = np.array([60000, 30000], np.int64)
    tp = np.array([10**6, 500], np.int64)
    gp = mad_gpu.MipsPlan.create(to_dev(A))
    res = gp.batch(to_dev(Q), s, tp, T, seed=SEED)
    for q in range(2):
        o, ok, ox, _ = _oracle_query(A, Q[q], q, s[q], tp[q], T)
        gk, gx, F = gp.query_scores(q)
        assert F == o["F"]
        assert np.array_equal(gk, ok) and np.array_equal(gx, ox)
        assert gk.max() >= m - 8  # the last rows' keys are in the table
        _check_query(A, q, Q[q], res[q], o, T)
    gp.close()

"""Benchmark: diamond sampling (Alg. 3 with Alg. 2) on one MI355X.

A step is one pass of the whole hot path over the resident inputs:
mad_plan_refresh (norms, stage weights, quanta, alias tables) followed by
mad_plan_topk (sampling into the score table X, top-t' selection, fp32
verification, top-t).  The default workload is dense A, B of 1e5 vectors in
d = 100 (N(0,1) fp32 with 50 planted pairs at |a.b| = 5 sqrt(d)),
s = 1e7 samples, t' = 1e4, t = 100.

Prints one JSON line.  value = samples per second of whole steps (inputs
already in HBM).  roofline = the sampling kernel's algorithmic bytes per
launch over its HIP-event duration.  cpu_baseline = the CPU oracle timed on
the host for the same step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one dense sample: three 8-byte alias entries (T1[k],
# T2[k], T3[i]; T0 sits in LDS) + the 4-byte fourth edge b_k'j, 28 bytes.
# The design also writes each sample's 12-byte pair (8-byte key, 4-byte
# signed fourth edge) for the score accumulation; that write is reported
# beside the roofline, not counted in it.
SAMPLE_READ_BYTES = 3 * 8 + 4
PAIR_WRITE_BYTES = 12
# worker processes of the all-cores oracle baseline (the host share of one
# GPU)
CPU_WORKERS_MAX = 16
# rows of A whose exhaustive top t the host computes for the CPU exact
# baseline (scaled to all m rows)
CPU_EXACT_ROWS = 4096
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sample_dense_traffic.json")
SAMPLER_SRC = os.path.join(ROOT, "paper_1506_03872_amd", "csrc",
                           "sampler.hip")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--bruteforce-only", action="store_true",
                    help="dense configs: only the MFMA brute force per "
                         "precision (ms, TFLOP/s, recall), one JSON line")
    ap.add_argument("--unit-values", action="store_true",
                    help="sparse configs: every stored value 1 (0/1 inputs)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the time-to-recall sweep")
    ap.add_argument("--no-sparse", action="store_true",
                    help="leave the sparse C3 summary out of the dense line")
    ap.add_argument("--binary", type=float, default=0.0,
                    help="dense configs: 0/1 inputs of the same shape with "
                         "this density (the binary inputs of Alg. 1)")
    ap.add_argument("--ceilings-sweep", action="store_true",
                    help="print the memory probe rates over buffers of "
                         "0.25 MB to 512 MB (one JSON line each) and exit")
    return ap.parse_args()


def sampler_src_hash():
    with open(SAMPLER_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(launch_samples):
    """HBM bytes per launch of the sampling kernel from the committed
    rocprofv3 counter summary (None when absent or stale)."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("sampler_src_sha256_16") != sampler_src_hash():
        return None
    if rec.get("samples_per_launch") != launch_samples:
        return None
    return rec.get("hbm_bytes_per_launch")


PROBE_KINDS = {0: "rand_load_8B", 1: "rand_load_4B", 2: "rand_atomic_add_8B",
               3: "rand_cas_8B", 4: "rand_cas_then_add_16B",
               5: "stream_copy_8B"}


def memory_ceilings(mad, footprint_words=1 << 26, nops=1 << 26, reps=3):
    """Operations per second of mad_probe_memory on a buffer of 512 MB
    (the size class of the sampler's tables and score table)."""
    import torch
    buf = torch.zeros(footprint_words, dtype=torch.int64, device="cuda")
    out = {}
    for kind, name in PROBE_KINDS.items():
        ops = nops if kind != 5 else footprint_words // 2
        mad.probe_memory(kind, buf, ops, seed=1)  # warm
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for r in range(reps):
            mad.probe_memory(kind, buf, ops, seed=2 + r)
        ev1.record()
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) * 1e-3 / reps
        out[name] = ops / sec / 1e9  # G operations per second
    out["stream_copy_GBps"] = out["stream_copy_8B"] * 16
    del buf
    return out


# dense MFMA peaks of MI355X (TFLOP/s), no sparsity
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}


def exact_topk_gpu(A, B, t):
    """Exhaustive top-t by |c| (FP64 products on the GPU, row blocks)."""
    import torch
    n = B.shape[0]
    B64T = B.double().t().contiguous()
    best_v = torch.empty(0, dtype=torch.float64, device=A.device)
    best_k = torch.empty(0, dtype=torch.int64, device=A.device)
    # torch.topk sorts at most INT_MAX elements: rows per block so that a
    # block holds at most 2^30 products
    blk = max(1, min(4096, (1 << 30) // n))
    for i0 in range(0, A.shape[0], blk):
        Cb = A[i0:i0 + blk].double() @ B64T
        v, idx = torch.topk(Cb.abs().flatten(), min(t, Cb.numel()))
        keys = (i0 + idx // n) * n + idx % n
        best_v = torch.cat([best_v, v])
        best_k = torch.cat([best_k, keys])
        v2, o = torch.topk(best_v, min(t, best_v.numel()))
        best_v, best_k = v2, best_k[o]
    return best_k.cpu().numpy(), best_v.cpu().numpy()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_range(job):
    """Worker of the all-cores oracle baseline: the closed samples of one
    range of l as (key, increment) arrays.  Each worker regenerates the
    seeded inputs and builds its own oracle tables (part of the timed work)."""
    import numpy as np
    import oracle
    import workloads
    config, data_seed, sample_seed, l0, cnt, F, binary = job
    cfg, data = workloads.make(config, seed=data_seed)
    if binary:
        A, B = workloads.binary(cfg["m"], cfg["n"], cfg["d"], binary,
                                seed=data_seed)
    else:
        A, B = data["A"], data["B"]
    p = oracle.Plan.dense(A, B)
    r = p.samples(sample_seed, l0, cnt, F)
    p.close()
    closed = r["inc"] != 0
    n = B.shape[0]
    return (r["i"][closed].astype(np.int64) * n + r["j"][closed],
            r["inc"][closed])


def cpu_baseline(A, B, cfg, args):
    """The oracle on the host for one whole step of the workload (tables, s
    samples, Alg. 2): once on one thread, once split over worker processes
    by ranges of l (each worker builds its tables; X is merged exactly)."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    seed = args.seed
    s, tp, t = cfg["s"], cfg["t_prime"], cfg["t"]
    t0 = time.perf_counter()
    p = oracle.Plan.dense(A, B)
    t1 = time.perf_counter()
    r1 = p.topk(seed=seed, s=s, t_prime=tp, t=t)
    t2 = time.perf_counter()
    one = t2 - t0
    ncpu = os.cpu_count() or 1
    workers = max(1, min(ncpu, CPU_WORKERS_MAX))
    F = p.fix_exponent(s)
    bounds = np.linspace(0, s, workers + 1).astype(np.int64)
    jobs = [(args.config, args.seed, seed, int(bounds[w]),
             int(bounds[w + 1] - bounds[w]), F, args.binary)
            for w in range(workers)]
    t3 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        parts = pool.map(_oracle_range, jobs)
    keys, x = oracle.merge_scores(parts)
    rw = p.post(keys, x, tp, t)
    t4 = time.perf_counter()
    p.close()
    allc = t4 - t3
    if not (np.array_equal(rw["key"], r1["key"]) and
            np.array_equal(rw["tp_key"], r1["tp_key"])):
        raise SystemExit("the split oracle run differs from the single one")
    # the exhaustive answer on the host, the paper's exact baseline (a CPU
    # BLAS product): the oracle's FP64 products in row blocks (numpy with
    # its BLAS on the host's cores) for the first rows of A, scaled to m
    m, d = A.shape
    n = B.shape[0]
    rows = min(m, CPU_EXACT_ROWS)
    t5 = time.perf_counter()
    oracle.exact_topk(A[:rows], B, t, block=256)
    ex = time.perf_counter() - t5
    exact = dict(kind="oracle exact_topk: FP64 products in row blocks "
                      "(numpy BLAS), top t by |c|",
                 rows=rows, seconds=round(ex, 3),
                 full_seconds_est=round(ex * m / rows, 2),
                 pairs_per_s=round(rows * n / ex, 1),
                 blas_threads=os.environ.get("OMP_NUM_THREADS", str(ncpu)))
    return dict(value=s / allc, unit="samples/s", cores=workers,
                kind="oracle",
                sample="one full step of the same workload (tables + s=%d "
                       "samples + Alg. 2): %d worker processes over ranges "
                       "of l, each building its own tables, X merged exactly "
                       "(%.2f s)" % (s, workers, allc),
                host_cpu_count=ncpu, cpu_model=cpu_model(),
                one_thread={"value": s / one, "seconds": round(one, 2),
                            "tables_seconds": round(t1 - t0, 2)},
                exact=exact), r1


# algorithmic bytes of one MIPS sample: the T1[k] and T3[i] alias entries
# (stage 0 and the query live in LDS), and for a closed sample one 8-byte
# score slot (key and x packed) read and written once
MIPS_SAMPLE_READ_BYTES = 2 * 8
MIPS_SCORE_RMW_BYTES = 2 * 8


def exact_topk_rows(A, Q, t, blk=256):
    """Per query: indices and |c| of the exact top t by |a_i . q| (FP64)."""
    import torch
    AT = A.double().t().contiguous()
    idx, val = [], []
    for q0 in range(0, Q.shape[0], blk):
        C = (Q[q0:q0 + blk].double() @ AT).abs_()
        v, i = torch.topk(C, t, dim=1)
        idx.append(i.cpu())
        val.append(v.cpu())
        del C
    return torch.cat(idx).numpy(), torch.cat(val).numpy()


def bench_mips(args, cfg, data, mad):
    import numpy as np
    import torch
    A_h, Q_h, s_q = data["A"], data["Q"], data["s_q"]
    tp_q = s_q.copy()  # dot-product budget t' = s per query (Sec. 6)
    t = cfg["t"]
    nq, d = Q_h.shape
    m = A_h.shape[0]
    A = torch.from_numpy(A_h).cuda()
    Q = torch.from_numpy(Q_h).cuda()
    plan = mad.MipsPlan.create(A)
    log("autotune")
    tuned = plan.autotune(Q, s_q, tp_q, t, seed=args.seed, reps=1)
    log("tuned %s" % tuned)
    out = torch.empty((nq * t, 3), dtype=torch.int64, device="cuda")
    n_out = torch.zeros(nq, dtype=torch.int64, device="cuda")
    for _ in range(args.warmup):
        plan.batch_raw(Q, s_q, tp_q, t, args.seed, out, n_out)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        plan.batch_raw(Q, s_q, tp_q, t, args.seed, out, n_out)
    ev1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    ms = ev0.elapsed_time(ev1) / args.steps
    st = plan.mips_stats(nq)
    ref_out, ref_n = out.clone(), n_out.clone()
    # the same batch with each verification precision (bf16 / fp8 screen
    # before fp32): ms per batch, fp32 rows read, identical results
    vprec = {}
    for name, prec in (("fp32", mad.MAD_FP32), ("bf16", mad.MAD_BF16),
                       ("fp8_e4m3", mad.MAD_FP8_E4M3)):
        plan.set_verify_precision(prec)
        plan.batch_raw(Q, s_q, tp_q, t, args.seed, out, n_out)
        torch.cuda.synchronize()
        e0v = torch.cuda.Event(enable_timing=True)
        e1v = torch.cuda.Event(enable_timing=True)
        e0v.record()
        for _ in range(args.steps):
            plan.batch_raw(Q, s_q, tp_q, t, args.seed, out, n_out)
        e1v.record()
        torch.cuda.synchronize()
        vs = plan.verify_stats()
        vprec[name] = {"ms_per_batch": round(e0v.elapsed_time(e1v) /
                                             args.steps, 3),
                       "n_cand": vs["n_cand"],
                       "n_reranked_fp32": vs["n_reranked"],
                       "same_result_as_fp32": bool(
                           torch.equal(n_out, ref_n) and
                           torch.equal(out, ref_out))}
        log("MIPS verify %s: %s" % (name, vprec[name]))
    plan.set_verify_precision(mad.MAD_FP32)
    # phase split from an eager run of the same batch
    tplan = mad.MipsPlan.create(A, flags=mad.MAD_FLAG_TIMING)
    tplan.set_config(tuned["chunk"], tuned["unroll"], tuned["grid"])
    tplan.set_table_factor(tuned["slots"])
    tplan.batch_raw(Q, s_q, tp_q, t, args.seed, out, n_out)
    tplan.batch_raw(Q, s_q, tp_q, t, args.seed, out, n_out)
    ph = tplan.phase_ms()
    tplan.close()
    S = int(s_q.sum())
    closed = st["closed"]
    alg = MIPS_SAMPLE_READ_BYTES * S + MIPS_SCORE_RMW_BYTES * closed
    achieved = alg / (ph[1] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": "k_sample_mips", "kernel_ms": round(ph[1], 4),
                "algorithmic_bytes_per_launch": alg}
    extra = {}
    if not args.no_recall:
        log("exact per-query top-%d" % t)
        ek, ev = exact_topk_rows(A, Q, t)
        cnt = n_out.cpu().numpy()
        raw = out.view(nq, t, 3).cpu().numpy()
        rec = []
        for q in range(nq):
            got = raw[q, :max(cnt[q], 0), 0]
            c64 = A_h[got].astype(np.float64) @ Q_h[q].astype(np.float64)
            rec.append(np.count_nonzero(np.abs(c64) >= ev[q, t - 1]) / t)
        extra["recall_at_10_mean"] = round(float(np.mean(rec)), 4)
        extra["queries_recall_ge_0.95"] = int(np.count_nonzero(
            np.array(rec) >= 0.95))
        # library brute force for context: fp32 GEMM + row top-t
        AT = A.t().contiguous()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for q0 in range(0, nq, 1024):
            C = (Q[q0:q0 + 1024] @ AT).abs_()
            torch.topk(C, t, dim=1)
            del C
        e1.record()
        torch.cuda.synchronize()
        extra["torch_fp32_gemm_topk_ms"] = round(e0.elapsed_time(e1), 3)
    # score updates against the probe ceiling of one CAS on a random 8-byte
    # word: a closed sample whose key is new claims a slot with key and
    # increment in one CAS; a key already present takes one more add, and a
    # probe past a taken slot one more CAS
    log("memory ceilings")
    ceil = memory_ceilings(mad)
    upd = closed / (ph[1] * 1e-3)
    cas = ceil["rand_cas_8B"] * 1e9
    distinct = int(st["distinct"])
    extra["score_updates"] = {
        "closed_per_s": round(upd, 1),
        "cas_ceiling_per_s": round(cas, 1),
        "frac_of_ceiling": round(upd / cas, 4),
        "adds_per_closed": round((closed - distinct) / max(closed, 1), 4),
        "note": "one CAS per closed sample (key and increment packed in one "
                "64-bit slot), plus an add when the key was already "
                "there; the kernel also makes two random alias-entry "
                "loads per sample, so it cannot reach this ceiling"}
    line = {
        "metric": "MIPS batch: diamond samples/s (queries/s, recall@10)",
        "value": round(S / (ms * 1e-3), 1),
        "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "wall_ms_per_step": round(wall, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+int64", "data": "synthetic",
        "config": {"workload": "mips_gaussian_%s" % args.config, "m": m,
                   "d": d, "nq": nq, "sum_s": S, "t": t,
                   "t_prime": "s per query", "seed": args.seed},
        "queries_per_s": round(nq / (ms * 1e-3), 1),
        "tuned": tuned,
        "phase_ms": {"query_tables": round(ph[0], 4),
                     "sample": round(ph[1], 4),
                     "postprocess": round(ph[2], 4),
                     "clear_scores": round(ph[3], 4)},
        "stats": {"closed": closed, "distinct": st["distinct"],
                  "n_pos_total": int(st["n_pos"].sum()),
                  "n_cand_total": int(st["n_cand"].sum())},
        "pairs_verified_per_s": round(float(st["n_cand"].sum()) /
                                      (ph[2] * 1e-3), 1),
        "verify_precision": vprec,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    line.update(extra)
    plan.close()
    print(json.dumps(line))


# bytes one sparse sample reads and writes: stage-0 entry (8 B, L2 resident
# for d = 1e5), the metas of T1[k] and T2[k] (8 B each), T1's and T2's
# 32-byte alias entries (with T3's meta of i and b_j's coordinate
# signature), T3's 16-byte entry, the 16-byte slot of B's entry table that
# holds b_jk' (counted for every sample, though the signature rules out
# most absent k' without it), then the 12-byte pair written
def csr_sample_bytes(nnz_per_vec):
    """Algorithmic bytes of one sparse sample (see above).  nnz_per_vec no
    longer enters: the fourth edge is one probe whatever the row's length."""
    del nnz_per_vec
    return 8 + 2 * 8 + 2 * 32 + 16 + 16 + PAIR_WRITE_BYTES


def bench_csr(args, cfg, data, mad):
    import numpy as np
    import torch
    a, b, m, n = data["a"], data["b"], data["m"], data["n"]
    if args.unit_values:
        a = (a[0], a[1], np.ones_like(a[2]))
        b = (b[0], b[1], np.ones_like(b[2]))
    d = cfg["d"]
    s, tp, t = cfg["s"], cfg["t_prime"], cfg["t"]
    ta = tuple(torch.from_numpy(x).cuda() for x in a)
    tb = tuple(torch.from_numpy(x).cuda() for x in b)
    log("plan (sparse tables)")
    t0 = time.perf_counter()
    plan = mad.Plan.csr(ta, tb, m, n, d, flags=mad.MAD_FLAG_TIMING)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    # creation validated the inputs; the timed refreshes skip the NaN / Inf
    # scan (the structure of the sparse inputs is checked on every build)
    plan.close()
    # timed steps without the phase events; a second plan with them for the
    # phase times
    plan = mad.Plan.csr(ta, tb, m, n, d, flags=mad.MAD_FLAG_NO_CHECK)
    out = torch.empty((t, 3), dtype=torch.int64, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")

    def step():
        plan.refresh()
        plan.topk_raw(t, s, tp, args.seed, out, n_out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    timed_out = out.clone()
    plan.close()
    plan = mad.Plan.csr(ta, tb, m, n, d,
                        flags=mad.MAD_FLAG_TIMING | mad.MAD_FLAG_NO_CHECK)
    step()
    torch.cuda.synchronize()
    if not torch.equal(out, timed_out):
        raise SystemExit("the timing plan's result differs from the timed one")
    phases = []
    for _ in range(min(args.steps, 5)):
        step()
        phases.append(plan.phase_ms())
    ph = np.array(phases)
    st = plan.stats()
    sampler_ms = float(ph[:, 1].mean())
    per = csr_sample_bytes(cfg["nnz"])
    alg = per * s
    achieved = alg / (sampler_ms * 1e-3) / 1e9
    amort = float(ph[:, 1].mean() + ph[:, 2].mean() + ph[:, 3].mean() +
                  ph[:, 4].mean())
    line = {
        "metric": "sparse diamond samples/s (whole step incl. table build)",
        "value": round(s / (ms_per_step * 1e-3), 1),
        "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+int64", "data": "synthetic",
        "config": {"workload": "powerlaw_csr_%s%s" % (
                       "unit_" if args.unit_values else "", args.config),
                   "m": m,
                   "n": n, "d": d, "nnz_per_vector": cfg["nnz"],
                   "zipf": cfg["zipf"], "s": s, "t_prime": tp, "t": t,
                   "seed": args.seed},
        "plan_create_ms": round(create_ms, 2),
        "amortized_samples_per_s": round(s / (amort * 1e-3), 1),
        "phase_ms": {"tables": round(float(ph[:, 0].mean()), 4),
                     "sample": round(sampler_ms, 4),
                     "accumulate": round(float(ph[:, 4].mean()), 4),
                     "postprocess": round(float(ph[:, 2].mean()), 4),
                     "clear_scores": round(float(ph[:, 3].mean()), 4)},
        "stats": {"wnorm": st["wnorm"], "closed": st["closed"],
                  "closure": round(st["closed"] / s, 5),
                  "distinct": st["distinct"], "n_pos": st["n_pos"],
                  "n_cand": st["n_cand"]},
        "pairs_verified_per_s": round(st["n_cand"] /
                                      (float(ph[:, 2].mean()) * 1e-3), 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": None, "kernel": "k_sample_csr",
                     "kernel_ms": round(sampler_ms, 4),
                     "algorithmic_bytes_per_launch": alg},
        "cpu_baseline": None,
    }
    plan.close()
    if not args.no_recall:
        line["recall"] = csr_recall(args, cfg, mad, a, b, m, n)
    print(json.dumps(line))


def csr_recall(args, cfg, mad, a, b, m, n, plan=None):
    """Threshold-recall@t of the sparse path at the full size against the
    exact sparse brute force (mad_bruteforce_topk_csr, bf16 certified
    filter, median of 3 runs): s on a x sqrt(10) grid, mean recall over
    seeds 0..4 and the median time of those top-k calls; time-to-recall
    end to end (plan build + top-k) and amortized (top-k only)."""
    import numpy as np
    import torch
    d, t, tp = cfg["d"], cfg["t"], cfg["t_prime"]
    ta = tuple(torch.from_numpy(x).cuda() for x in a)
    tb = tuple(torch.from_numpy(x).cuda() for x in b)
    times, res, st = [], None, None
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, st = mad.bruteforce_topk_csr(ta, tb, m, n, d, t,
                                          precision=mad.MAD_BF16)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    bf_ms = float(np.median(times))
    if len(res["c"]) < t:
        raise SystemExit("the exact sparse result has fewer than t pairs")
    tau = float(np.abs(res["c"].cpu().numpy()).min())
    log("sparse exact top-%d: %.1f ms (heavy %d, light wedges %d), tau %.2f"
        % (t, bf_ms, st["heavy"], st["light_wedges"], tau))
    own = plan is None
    # end to end counts a plan created from the inputs (transposes, layouts
    # and tables); a plan that already exists only rebuilds its tables
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fresh = mad.Plan.csr(ta, tb, m, n, d, flags=mad.MAD_FLAG_NO_CHECK)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    if own:
        plan = fresh
    else:
        fresh.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.refresh()
    torch.cuda.synchronize()
    refresh_ms = (time.perf_counter() - t0) * 1e3
    sweep, hit, stop = [], None, None
    # what torch's allocator holds from the dense part goes back to the
    # device, so that the largest s can have its workspace
    torch.cuda.empty_cache()
    s = 10 ** 6
    while True:
        try:
            plan.topk(t=t, s=s, t_prime=tp, seed=0)
        except mad.MadError as err:
            stop = "s = %d: workspace allocation failed (%s)" % (s, err)
            break
        recs, tms = [], []
        for seed in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = plan.topk(t=t, s=s, t_prime=tp, seed=seed)
            torch.cuda.synchronize()
            tms.append((time.perf_counter() - t0) * 1e3)
            # the returned c are fp32 sparse dot products, as the
            # brute force's: recall by threshold on them
            recs.append(float(np.count_nonzero(
                np.abs(r["c"].cpu().numpy()) >= tau)) / t)
        pt = {"s": s, "recall_at_t": round(float(np.mean(recs)), 4),
              "ms_topk": round(float(np.median(tms)), 3)}
        sweep.append(pt)
        log("sparse recall s=%d: %.3f (%.2f ms)" % (s, pt["recall_at_t"],
                                                   pt["ms_topk"]))
        if pt["recall_at_t"] >= 0.95:
            hit = pt
            stop = "recall 0.95 reached"
            break
        if pt["ms_topk"] > bf_ms:
            stop = ("top-k time %.1f ms > the exact brute force (%.1f ms)"
                    % (pt["ms_topk"], bf_ms))
            break
        nxt = int(round(s * 10 ** 0.5))
        # workspace of the next s (pairs and the accumulation's partition,
        # which the selection's boundary lists reuse, and the score table:
        # about 44 bytes per sample): stay below 200 GiB of the GPU's
        # 288 GB; past the last grid point that fits, one more point at the
        # largest s that does
        s_max = int((200 << 30) / 44) // 10 ** 8 * 10 ** 8
        if nxt > s_max:
            if s < 0.9 * s_max:
                nxt = s_max
            else:
                stop = ("next s = %d would need about %.0f GiB of workspace "
                        "(cap 200 GiB); last top-k %.1f ms, exact brute "
                        "force %.1f ms" % (nxt, 44 * nxt / 2 ** 30,
                                           pt["ms_topk"], bf_ms))
                break
        s = nxt
    if own:
        plan.close()
    return {"m": m, "n": n, "d": d, "t": t, "t_prime": tp, "tau": tau,
            "seeds": [0, 1, 2, 3, 4],
            "exact": "mad_bruteforce_topk_csr (heavy coordinates through "
                     "the bf16 certified MFMA brute force, light wedges "
                     "listed), median of 3",
            "exact_bruteforce_ms": round(bf_ms, 1),
            "exact_stats": {k: (round(v, 3) if isinstance(v, float) else v)
                            for k, v in st.items()},
            "plan_build_ms": round(build_ms, 2),
            "plan_refresh_ms": round(refresh_ms, 2),
            "time_to_recall_0.95": None if hit is None else {
                "s": hit["s"], "ms_topk": hit["ms_topk"],
                "ms_end_to_end": round(build_ms + hit["ms_topk"], 3),
                "ms_amortized": round(refresh_ms + hit["ms_topk"], 3),
                "speedup_vs_exact_end_to_end": round(
                    bf_ms / (build_ms + hit["ms_topk"]), 1)},
            "stop_rule": "s grows by sqrt(10) from 1e6 until recall reaches "
                         "0.95, a top-k call takes longer than the exact "
                         "brute force, or the workspace cap (200 GiB) or "
                         "the device memory is reached; the last point is "
                         "the largest s within the cap",
            "stop_reason": stop,
            "sweep": sweep}


def sparse_summary(args, mad):
    """The sparse workload (C3 at full size) inside the default line: one
    timed whole step at its s, and recall / time-to-recall against the
    exact sparse brute force."""
    import numpy as np
    import torch
    import workloads
    log("generating C3 (sparse)")
    cfg, data = workloads.make("C3", seed=args.seed)
    a, b, m, n = data["a"], data["b"], data["m"], data["n"]
    d, s, tp, t = cfg["d"], cfg["s"], cfg["t_prime"], cfg["t"]
    ta = tuple(torch.from_numpy(x).cuda() for x in a)
    tb = tuple(torch.from_numpy(x).cuda() for x in b)
    plan = mad.Plan.csr(ta, tb, m, n, d)
    plan.close()
    plan = mad.Plan.csr(ta, tb, m, n, d, flags=mad.MAD_FLAG_NO_CHECK)
    out = torch.empty((t, 3), dtype=torch.int64, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")

    def step():
        plan.refresh()
        plan.topk_raw(t, s, tp, args.seed, out, n_out)

    step()
    torch.cuda.synchronize()
    steps = 5
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    log("sparse C3 step %.2f ms" % ms)
    rec = csr_recall(args, cfg, mad, a, b, m, n, plan=plan)
    plan.close()
    return {"workload": "powerlaw_csr_C3", "m": m, "n": n, "d": d,
            "nnz_per_vector": cfg["nnz"], "s": s, "t_prime": tp, "t": t,
            "ms_per_step": round(ms, 3),
            "samples_per_s": round(s / (ms * 1e-3), 1),
            "recall": rec}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not "
              "supported (the score table and the selection would shard by "
              "a hash of (i, j); that path is not built)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1506_03872_amd as mad
    import workloads

    if args.ceilings_sweep:
        for lw in (15, 18, 21, 23, 25, 26):
            r = memory_ceilings(mad, footprint_words=1 << lw)
            print(json.dumps({"footprint_MB": (8 << lw) / 2**20,
                              "G_ops_per_s": {k: round(v, 2)
                                              for k, v in r.items()}}),
                  flush=True)
        return
    log("generating %s" % args.config)
    cfg, data = workloads.make(args.config, seed=args.seed)
    if cfg["kind"] == "mips":
        bench_mips(args, cfg, data, mad)
        return
    if cfg["kind"] == "csr":
        bench_csr(args, cfg, data, mad)
        return
    if cfg["kind"] not in ("dense", "planted", "planted_wide"):
        print("bench.py: config %s is not a dense MAD workload" % args.config,
              file=sys.stderr)
        sys.exit(2)
    A_h, B_h = data["A"], data["B"]
    if args.binary:
        A_h, B_h = workloads.binary(A_h.shape[0], B_h.shape[0], A_h.shape[1],
                                    args.binary, seed=args.seed)
        data = {"A": A_h, "B": B_h}
    s, tp, t = cfg["s"], cfg["t_prime"], cfg["t"]
    dev = torch.device("cuda:0")
    A = torch.from_numpy(A_h).to(dev)
    B = torch.from_numpy(B_h).to(dev)
    m, d = A.shape
    n = B.shape[0]
    # the inputs are validated once here; the timed plan skips the per-call
    # NaN / Inf check (and the host synchronisation that reports it)
    if not (bool(torch.isfinite(A).all()) and bool(torch.isfinite(B).all())):
        raise SystemExit("synthetic inputs hold NaN or Inf")
    if args.bruteforce_only:
        # the MFMA brute force alone, per precision, on this workload
        recall_of, c_error = recall_helpers(A, B, A_h, B_h, t)
        bf = bruteforce_report(mad, A, B, t, recall_of, c_error)
        print(json.dumps({"workload": "dense_planted_%s" % args.config,
                          "m": m, "n": n, "d": d, "t": t,
                          "bruteforce": bf}), flush=True)
        return
    # the timed steps run on a plan without phase events (each event is a
    # marker on the stream, about 2% of a C2 step); a second plan with them
    # then gives the phase times and the sampling kernel's time
    plan = mad.Plan.dense(A, B, flags=mad.MAD_FLAG_NO_CHECK)
    out = torch.empty((t, 3), dtype=torch.int64, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)

    def step():
        plan.refresh()
        plan.topk_raw(t, s, tp, args.seed, out, n_out)

    log("plan built; warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    timed_out = out.clone()
    plan.close()
    plan = mad.Plan.dense(A, B,
                          flags=mad.MAD_FLAG_TIMING | mad.MAD_FLAG_NO_CHECK)
    step()
    torch.cuda.synchronize()
    if not torch.equal(out, timed_out):
        raise SystemExit("the timing plan's result differs from the timed one")
    # phase times from the plan's events, in steps of their own (reading
    # them synchronises every step)
    phases = []
    for _ in range(min(args.steps, 5)):
        step()
        phases.append(plan.phase_ms())
    ph = np.array(phases)
    # the roofline kernel: k_sample_dense alone (after the k-order passes)
    sampler_ms = float(ph[:, 5].mean())
    sampling_ms = float(ph[:, 1].mean())
    stats = plan.stats()
    res = mad.unpack_pairs(out, int(n_out.item()))

    closed = stats["closed"]
    alg_bytes = SAMPLE_READ_BYTES * s
    achieved = alg_bytes / (sampler_ms * 1e-3) / 1e9
    traffic = measured_traffic(s)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": traffic,
                "kernel": "k_sample_dense",
                "kernel_ms": round(sampler_ms, 4),
                "algorithmic_bytes_per_launch": alg_bytes,
                "algorithmic_bytes_per_sample": SAMPLE_READ_BYTES,
                "pair_write_bytes_per_launch": PAIR_WRITE_BYTES * s}

    log("%.3f ms/step" % ms_per_step)
    log("memory ceilings")
    ceil = memory_ceilings(mad)
    if traffic:
        roofline["traffic_GBps"] = round(traffic / (sampler_ms * 1e-3) / 1e9,
                                         1)
        roofline["traffic_frac_of_peak"] = round(
            roofline["traffic_GBps"] / HBM_PEAK_GBS, 4)
        roofline["traffic_bytes_per_sample"] = round(traffic / s, 1)
    # reference rates of uniform random accesses over a 512 MB buffer (not a
    # bound of the sampler, whose ordered draws hit L2 and the MALL)
    roofline["random_access_reference_Gops"] = {
        k: round(v, 3) for k, v in ceil.items()}
    extra = {}
    if not args.no_recall:
        recall_of, c_error = recall_helpers(A, B, A_h, B_h, t)
        rec, keys = recall_of(res["i"].cpu().numpy(), res["j"].cpu().numpy())
        extra["recall_at_t"] = rec
        if "planted_i" in data:
            pk = set((data["planted_i"] * n + data["planted_j"]).tolist())
            extra["planted_found"] = len(pk & set(keys.tolist()))
            extra["planted_total"] = len(pk)
        extra["verify_precision"] = verify_precisions(
            args, mad, plan, step, out, n_out, recall_of, c_error, A_h, B_h,
            tp)
        extra["bruteforce"] = bruteforce_report(mad, A, B, t, recall_of,
                                                c_error)
        if not args.no_sweep:
            extra["time_to_recall"] = time_to_recall(
                args, mad, plan, A, B, t, tp, recall_of, extra["bruteforce"])
    plan.close()
    base = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        base, _ = cpu_baseline(A_h, B_h, cfg, args)
    if not args.no_recall and not args.no_sparse and not args.binary:
        del A, B
        torch.cuda.empty_cache()
        extra["sparse_C3"] = sparse_summary(args, mad)

    line = {
        "metric": "diamond samples/s + time-to-recall@0.95 vs MFMA brute "
                  "force, 1 MI355X",
        "value": round(s / (ms_per_step * 1e-3), 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+int64",
        "data": "synthetic",
        "config": {"workload": ("dense_binary%g_%s" % (args.binary,
                                                          args.config)
                                if args.binary else
                                "dense_planted_%s" % args.config),
                   "m": m, "n": n, "d": d, "s": s, "t_prime": tp, "t": t,
                   "n_planted": int(len(data.get("planted_i", []))),
                   "seed": args.seed},
        "phase_ms": {"tables": round(float(ph[:, 0].mean()), 4),
                     "sample": round(sampling_ms, 4),
                     "k_order": round(sampling_ms - sampler_ms, 4),
                     "sample_kernel": round(sampler_ms, 4),
                     "accumulate": round(float(ph[:, 4].mean()), 4),
                     "postprocess": round(float(ph[:, 2].mean()), 4),
                     "clear_scores": round(float(ph[:, 3].mean()), 4)},
        "stats": {"wnorm": stats["wnorm"], "closed": closed,
                  "distinct": stats["distinct"], "n_pos": stats["n_pos"],
                  "n_cand": stats["n_cand"]},
        # closed diamonds per second of the sampling kernel, and candidates
        # verified per second of Alg. 2 (selection + verification + top t)
        "closed_per_s": round(closed / (sampler_ms * 1e-3), 1),
        "pairs_verified_per_s": round(
            stats["n_cand"] / (float(ph[:, 2].mean()) * 1e-3), 1),
        "roofline": roofline,
        "cpu_baseline": base,
    }
    line.update(extra)
    print(json.dumps(line))


def verify_precisions(args, mad, plan, step, out, n_out, recall_of,
                      c_error, A_h, B_h, tp):
    """Whole steps under each verification precision of Alg. 2 (fp32 rows
    for every candidate, or bf16 / fp8 screening with error bounds first):
    ms per step, candidates re-ranked in fp32, and whether the top-t is the
    same pair list as under fp32 verification."""
    import numpy as np
    import torch
    res = {}
    ref = None
    for name, prec in (("fp32", mad.MAD_FP32), ("bf16", mad.MAD_BF16),
                       ("fp8_e4m3", mad.MAD_FP8_E4M3)):
        plan.set_verify_precision(prec)
        step()
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 5))
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        got = out[:int(n_out.item())].cpu().numpy().copy()
        vs = plan.verify_stats()
        r = mad.unpack_pairs(out, int(n_out.item()))
        i_arr, j_arr = r["i"].cpu().numpy(), r["j"].cpu().numpy()
        rec, _ = recall_of(i_arr, j_arr)
        if ref is None:
            ref = got
        res[name] = {"ms_per_step": round(ms, 3), "n_cand": vs["n_cand"],
                     "n_reranked_fp32": vs["n_reranked"], "recall_at_t": rec,
                     "max_rel_err_c_vs_fp64": c_error(
                         i_arr, j_arr, r["c"].cpu().numpy()),
                     "same_top_t_as_fp32": bool(np.array_equal(got, ref))}
        if prec != mad.MAD_FP32:
            res[name]["screen"] = screen_error(plan, A_h, B_h, [tp])
        log("verify %s: %.2f ms, %d of %d candidates re-ranked in fp32" %
            (name, ms, vs["n_reranked"], vs["n_cand"]))
    plan.set_verify_precision(mad.MAD_FP32)
    return res


def screen_error(plan, A_h, B_h, plan_tp):
    """The low-precision screen values c^ of the last call's candidates
    against FP64, next to their a-priori bounds (margin >= |c^ - c_fp32|,
    and |c_fp32 - c| is far smaller)."""
    import numpy as np
    import torch
    xk, xx, _ = plan.scores()            # Omega_t': the top t' of X
    pos = xx > 0
    keys = xk[pos][np.lexsort((xk[pos], -xx[pos]))][:plan_tp[0]]
    n = B_h.shape[0]
    ch, mg = plan.lowp_screen(torch.from_numpy(keys).cuda())
    i, j = keys // n, keys % n
    c64 = (A_h[i].astype(np.float64) * B_h[j].astype(np.float64)).sum(1)
    err = np.abs(ch.astype(np.float64) - c64)
    ratio = err / np.maximum(mg.astype(np.float64), 1e-300)
    return {"pairs": int(len(keys)),
            "max_abs_err_vs_fp64": float(err.max()) if len(err) else None,
            "max_rel_err_vs_fp64": float((err / np.abs(c64)).max())
            if len(err) else None,
            "median_bound": float(np.median(mg)) if len(mg) else None,
            "max_err_over_bound": float(ratio.max()) if len(err) else None,
            "median_err_over_bound": float(np.median(ratio))
            if len(err) else None}


def recall_helpers(A, B, A_h, B_h, t):
    """recall_of(i, j): the share of the exact top t's threshold that the
    pairs reach (with their keys); c_error(i, j, c): the largest relative
    error of reported dot products against FP64."""
    import numpy as np
    n = B_h.shape[0]
    log("exact top-t for recall")
    ek, ev = exact_topk_gpu(A, B, t)
    tau = float(np.sort(ev)[::-1][t - 1])

    def recall_of(i_arr, j_arr):
        keys = i_arr * n + j_arr
        c64 = (A_h[keys // n].astype(np.float64) *
               B_h[keys % n].astype(np.float64)).sum(1)
        return float(np.count_nonzero(np.abs(c64) >= tau)) / t, keys

    def c_error(i_arr, j_arr, c_arr):
        """largest |c - c64| / |c64| of reported dot products"""
        if len(i_arr) == 0:
            return None
        c64 = (A_h[i_arr].astype(np.float64) *
               B_h[j_arr].astype(np.float64)).sum(1)
        err = np.abs(c_arr.astype(np.float64) - c64) / np.maximum(
            np.abs(c64), 1e-300)
        return float(err.max())

    return recall_of, c_error


def bruteforce_report(mad, A, B, t, recall_of, c_error):
    """The MFMA brute force of the same top-t in each precision (median of
    5 runs): ms, recall@t, candidates re-ranked in fp32, and the largest
    relative error of its reported c against FP64."""
    import numpy as np
    import torch
    bf = {}
    for name, prec, ts in (("fp32", mad.MAD_FP32, 0),
                           ("bf16", mad.MAD_BF16, 0),
                           ("bf16_screen", mad.MAD_BF16, 20 * t),
                           ("fp8_screen", mad.MAD_FP8_E4M3, 20 * t)):
        times = []
        for r in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, st = mad.bruteforce_topk(A, B, t, precision=prec,
                                          t_screen=ts)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        i_arr, j_arr = res["i"].cpu().numpy(), res["j"].cpu().numpy()
        rec, _ = recall_of(i_arr, j_arr)
        ms = float(np.median(times))
        # algorithmic 2 m n d flops against the dense MFMA peak of the
        # precision the GEMM runs in
        tflops = 2.0 * A.shape[0] * B.shape[0] * A.shape[1] / (ms * 1e-3) / 1e12
        peak = {"fp32": MFMA_PEAK_TFLOPS["fp32"],
                "bf16": MFMA_PEAK_TFLOPS["bf16"],
                "bf16_screen": MFMA_PEAK_TFLOPS["bf16"],
                "fp8_screen": MFMA_PEAK_TFLOPS["fp8"]}[name]
        bf[name] = {"ms": round(ms, 3),
                    "tflops": round(tflops, 1),
                    "mfma_frac": round(tflops / peak, 4),
                    "recall": rec, "candidates": st["candidates"],
                    "max_rel_err_c_vs_fp64": c_error(
                        i_arr, j_arr, res["c"].cpu().numpy())}
        log("brute force %s: %.2f ms recall %.3f" % (name, bf[name]["ms"], rec))
    return bf


def time_to_recall(args, mad, plan, A, B, t, tp, recall_of, bf,
                   target=0.95, seeds=5):
    """Median wall time of whole steps (tables + sampling + Alg. 2) to reach
    mean threshold-recall@t >= target over `seeds` seeds, s on a x sqrt(10)
    grid, against the MFMA brute force (median of 5).  The sweep stops when
    a step takes 10x the fp32 brute force."""
    import numpy as np
    import torch
    limit = 10 * bf["fp32"]["ms"]
    out = torch.empty((t, 3), dtype=torch.int64, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    sweep, reached = [], None
    s = 100_000
    while True:
        recs, walls, amort = [], [], []
        for seed in range(seeds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.refresh()
            plan.topk_raw(t, s, tp, seed, out, n_out)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
            ph = plan.phase_ms()
            amort.append(ph[1] + ph[2] + ph[3] + ph[4])
            r = mad.unpack_pairs(out, int(n_out.item()))
            recs.append(recall_of(r["i"].cpu().numpy(),
                                  r["j"].cpu().numpy())[0])
        pt = {"s": s, "recall_mean": round(float(np.mean(recs)), 4),
              "ms_end_to_end": round(float(np.median(walls)), 3),
              "ms_amortized": round(float(np.median(amort)), 3)}
        sweep.append(pt)
        log("sweep s=%d recall %.3f %.2f ms" % (s, pt["recall_mean"],
                                                pt["ms_end_to_end"]))
        if pt["recall_mean"] >= target:
            reached = pt
            stop = "recall %.2f reached" % target
            break
        nxt = int(round(s * 10 ** 0.5))
        if pt["ms_end_to_end"] > limit:
            stop = ("step time %.1f ms > 10x the fp32 brute force (%.1f ms)"
                    % (pt["ms_end_to_end"], limit))
            break
        # workspace of the next s (pairs, partition, score table, about 64
        # bytes per sample): stay below 64 GiB
        if 64 * nxt > (64 << 30):
            stop = ("next s = %d would need about %.0f GiB of workspace "
                    "(cap 64 GiB); last step %.1f ms, 10x brute force is "
                    "%.1f ms" % (nxt, 64 * nxt / 2 ** 30,
                                 pt["ms_end_to_end"], limit))
            break
        s = nxt
    best = max(sweep, key=lambda p: p["recall_mean"])
    return {"target": target, "seeds": seeds, "t_prime": tp,
            "reached": reached is not None,
            "s_at_target": reached["s"] if reached else None,
            "ms_at_target": reached["ms_end_to_end"] if reached else None,
            "ms_at_target_amortized": (reached["ms_amortized"]
                                       if reached else None),
            "best_recall": best["recall_mean"], "best_s": best["s"],
            "stop_rule": "stop when recall reaches the target, a step takes "
                         "10x the fp32 brute force, or the workspace cap is "
                         "reached",
            "stop_reason": stop,
            "sweep": sweep}


if __name__ == "__main__":
    main()

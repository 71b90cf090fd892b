/*
 * mad.h -- C ABI of the MI355X (gfx950) diamond-sampling library.
 *
 * Problem (Ballard, Kolda, Pinar, Seshadhri, "Diamond Sampling for
 * Approximate Maximum All-pairs Dot-product (MAD) Search", Definition 1):
 * given vectors a_1..a_m and b_1..b_n in R^d, find the t pairs (i, j) with
 * the largest |a_i . b_j|.  The library runs diamond sampling (Alg. 3) and
 * its postprocessing (Alg. 2) on one GPU, plus an exhaustive brute force.
 *
 * Conventions for every entry point:
 *  - Layout: vectors are ROWS.  A is m x d row-major fp32 (a_i = A[i*d ..]),
 *    B is n x d row-major fp32.  This is the same memory as the paper's
 *    column-vector d x m matrices (Sec. 2).
 *  - Pointers marked (device) are device memory on the current HIP device;
 *    (host) pointers are host memory.  The caller owns every array it passes.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls enqueue their work on it and return without waiting, except where
 *    a call says it synchronises.
 *  - Return value: MAD_OK or a negative MAD_E* code; mad_last_error() then
 *    describes the failure (thread-local).  No exception crosses the ABI.
 *  - Results are a deterministic function of the inputs, t, s, t' and seed:
 *    the sampler draws sample l from the Philox4x64-10 block with counter
 *    (l, query, 0, 0) and key (seed, 0), and scores are exact int64 fixed
 *    point, so launch shapes and atomics ordering never change a result.
 */
#ifndef MAD_H
#define MAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One result pair.  c = a_i . b_j computed in fp32 (the verification of
 * Alg. 2);
 * x = the sampler's score x_ij (the score update of Alg. 3) converted to fp32. */
typedef struct mad_pair {
  int64_t i;
  int64_t j;
  float c;
  float x;
} mad_pair;

enum {
  MAD_OK = 0,
  MAD_EINVAL = -1,       /* bad argument (shape, pointer, t' < t, NaN/Inf) */
  MAD_ENOMEM = -2,       /* device allocation failed                       */
  MAD_EHIP = -3,         /* a HIP runtime call failed                      */
  MAD_EOVERFLOW = -4,    /* an internal capacity was exceeded              */
  MAD_EUNSUPPORTED = -5  /* option not available                           */
};

/* Arithmetic of the exhaustive brute force (mad_bruteforce_topk). */
enum { MAD_FP32 = 0, MAD_BF16 = 1, MAD_FP8_E4M3 = 2 };

/* Plan flags. */
enum {
  MAD_FLAG_NONE = 0,
  /* skip the NaN/Inf check of the inputs.  For sparse plans the caller
   * also vouches that the sparsity structure (pointers and coordinates)
   * stays the one of the plan's first build, which is checked: later
   * builds reuse its transposes and table layouts and only regather the
   * values.  Builds then never synchronise with the host. */
  MAD_FLAG_NO_CHECK = 1u << 0,
  MAD_FLAG_TIMING = 1u << 1,   /* record HIP events around each phase      */
  /* Gram matrix (Sec. 3.2.2, equal inputs): B must be A (same arrays, n = m).
   * The scores are symmetrised before Alg. 2, X <- (X + X^T) / 2, kept as
   * the exact sum x_ij + x_ji under the pair with i < j, and the diagonal
   * (a vector with itself) is left out, as in the paper's A^T A
   * experiments; results list pairs with i < j and report x = (x_ij +
   * x_ji) / 2. */
  MAD_FLAG_GRAM = 1u << 2,
  /* Squared matrix (Sec. 3.2.3, equal symmetric inputs): B must be A (same
   * arrays) with m = n = d and A == A^T (checked unless MAD_FLAG_NO_CHECK;
   * MAD_EINVAL otherwise), so C = A^2.  Every closed three-path also adds
   * its increment to x_kk' (the paper adds half to x_ij and half to x_kk'),
   * then the scores are symmetrised and the diagonal is left out as with
   * MAD_FLAG_GRAM, which this flag implies.  The kept score of i < j is
   * 2 (x_ij + x_ji) in those full increments; results report x as the
   * symmetrised entry of the paper, (x_ij + x_ji) / 2 with half
   * increments.  F is taken for 2s updates.  X is built from pairs only
   * (MAD_OPT_ACCUM = MAD_ACCUM_HASH is MAD_EUNSUPPORTED) and the sampler
   * runs in k order at most. */
  MAD_FLAG_SQUARE = 1u << 3
};

typedef struct mad_plan mad_plan;

/* ---------------------------------------------------------------------------
 * mad_plan_create_dense -- preprocessing of Alg. 3 (the weights w_ki and the
 * cumulative tables of Sec. 3.3 "Preprocessing" / Sec. 5.2) for dense A, B.
 *
 * Builds, in FP64 on the GPU, na_i = ||a_i||_1, nb_k = ||B_k*||_1,
 * v_k = sum_i |a_ki| na_i and the stage weights nb_k v_k (their total is
 * ||W||_1 with w_ki = |a_ki| ||a_i||_1 ||B_k*||_1), then one alias table per
 * stage distribution: T0 over k (weight nb_k v_k), T1[k] over i (weight
 * |a_ki| na_i), T2[k] over j (weight |b_kj|), T3[i] over k' (weight |a_k'i|).
 *   A (device) m x d fp32, B (device) n x d fp32; 1 <= m, n < 2^31, d >= 1.
 *   The plan BORROWS A and B: they must stay allocated and unchanged until
 *   mad_plan_destroy (mad_plan_refresh re-reads them after a change).
 *   flags: MAD_FLAG_*.  *plan (host) receives the new plan.
 * Allocates device memory and synchronises `stream` once (to report
 * non-finite inputs as MAD_EINVAL).
 * ------------------------------------------------------------------------- */
int mad_plan_create_dense(const float* A, int64_t m, const float* B,
                          int64_t n, int64_t d, uint32_t flags, void* stream,
                          mad_plan** plan);

/* ---------------------------------------------------------------------------
 * mad_plan_create_csr -- the same preprocessing for sparse vectors given as
 * compressed rows of the vector-major arrays: vector i of A has entries
 * a_idx[a_ptr[i] .. a_ptr[i+1]) (coordinates, strictly increasing, in
 * [0, d)) with values a_val[...]; likewise B.  All arrays (device);
 * ptr arrays hold m+1 (n+1) int64 entries.  Borrowed like the dense form.
 * Returns MAD_EINVAL for unsorted/duplicate/out-of-range coordinates.
 * ------------------------------------------------------------------------- */
int mad_plan_create_csr(const int64_t* a_ptr, const int32_t* a_idx,
                        const float* a_val, int64_t m, const int64_t* b_ptr,
                        const int32_t* b_idx, const float* b_val, int64_t n,
                        int64_t d, uint32_t flags, void* stream,
                        mad_plan** plan);

/* Rebuild every table of `plan` from the (same-shaped) borrowed inputs,
 * e.g. after their contents changed.  No allocation; synchronises once
 * unless the plan was made with MAD_FLAG_NO_CHECK.  A checked sparse plan
 * re-validates and re-transposes the inputs; an unchecked one keeps the
 * structure of its first build (values may change, the sparsity pattern
 * may not). */
int mad_plan_refresh(mad_plan* plan, void* stream);

/* ---------------------------------------------------------------------------
 * mad_plan_topk -- Alg. 3 sampling loop + Alg. 2 postprocessing.
 *   s        number of three-path samples (Alg. 3 loop over l), s >= 0
 *   t_prime  budget of exact dot products (Alg. 2), t_prime >= t
 *   t        number of pairs returned, t >= 1, t <= m*n
 *   seed     Philox key word 0
 *   out      (device) capacity t, filled in order of |c| descending, then
 *            (i, j) ascending
 *   n_out    (device) one int64: number of pairs written (<= t; fewer when
 *            fewer than t pairs have a positive score, Alg. 2)
 * Scores: x_ij accumulates sgn(a_ki b_kj a_k'i) b_k'j as int64 fixed point
 * with 2^F units, F = 62 - e - ceil(log2 max(s, 2)) where max|b| < 2^e.
 * Candidates are the pairs with x_ij > 0, the top t' of them by x
 * (ties by (i, j) ascending) are verified with fp32 dot products.
 * The first call for a given size allocates workspace; later calls with
 * the same or smaller (s, t', t) neither allocate nor synchronise.  The
 * workspace grows with s (score table, per-sample pairs, candidate lists)
 * and holds up to 32 MiB more for refining a long boundary of tied scores.
 * ------------------------------------------------------------------------- */
int mad_plan_topk(mad_plan* plan, int64_t t, int64_t s, int64_t t_prime,
                  uint64_t seed, mad_pair* out, int64_t* n_out, void* stream);

/* ---------------------------------------------------------------------------
 * mad_plan_set_verify_precision -- arithmetic of the verification of Alg. 2
 * for later mad_plan_topk calls on a dense plan:
 *   MAD_FP32      (default) fp32 dot products of every candidate;
 *   MAD_BF16, MAD_FP8_E4M3  every candidate is first computed from bf16 /
 *                 fp8-e4m3 copies of A and B (per-vector power-of-two scale
 *                 for fp8, fp32 accumulation) together with an a-priori
 *                 bound on its error (input rounding, fp32 accumulation of
 *                 d terms and the fp32 re-rank's own error; Higham,
 *                 "Accuracy and Stability of Numerical Algorithms", Sec. 3.1);
 *                 only candidates whose upper bound reaches the t-th largest
 *                 lower bound are verified in fp32.  The result is the same
 *                 as with MAD_FP32, with fewer fp32 rows read.
 * Builds the copies (device memory, kept in the plan and rebuilt by
 * mad_plan_refresh).  On a MIPS plan the same screen applies to each
 * query's candidates in mips_topk_batch (the database copy is built here,
 * the queries' copies in every batch).  MAD_EUNSUPPORTED for sparse plans.
 * ------------------------------------------------------------------------- */
int mad_plan_set_verify_precision(mad_plan* plan, int precision, void* stream);

/* Candidates of the last mad_plan_topk (host outputs, synchronises):
 * n_cand = |Omega_t'|, n_reranked = how many were verified in fp32 (equal
 * to n_cand under MAD_FP32 verification); on a MIPS plan, both summed over
 * the queries of the last batch.  Either pointer may be NULL. */
int mad_plan_verify_stats(mad_plan* plan, int64_t* n_cand,
                          int64_t* n_reranked);

/* ---------------------------------------------------------------------------
 * Launch choices of a MAD plan.  None changes a result: scores are exact
 * int64 sums, so X, the candidates and the output are the same under every
 * setting; they exist for measurement and for tests of each code path.
 *   MAD_OPT_ACCUM          how X (the score update of Alg. 3) is built:
 *                          MAD_ACCUM_PAIRS (default): every sample writes
 *                          its (key, signed fourth edge) pair and the pairs
 *                          are summed per key after a hash partition;
 *                          MAD_ACCUM_HASH: the sampler adds each increment
 *                          into an open-addressing table with int64 atomics.
 *                          Dense and sparse plans.
 *   MAD_OPT_SAMPLER_ORDER  dense plans, d <= 1024: 1 (default) draws the
 *                          samples grouped by their stage-0 coordinate k
 *                          (the first reordering of Sec. 5.2); 2 also
 *                          reorders them by i for the k' draw and by j for
 *                          the fourth edge (the whole scheme of Sec. 5.2;
 *                          pair form of X only, else it runs as 1); 0 draws
 *                          them in index order.
 *   MAD_OPT_ORDER_CHUNK    dense plans: samples per ordering pass, a power
 *                          of two in [2^12, 2^28] (default 2^28); longer
 *                          runs are ordered in consecutive chunks.
 * The process defaults come from the environment (MAD_ACCUM=hash,
 * MAD_SAMPLER_ORDER=0).  A change takes effect at the next mad_plan_topk,
 * which then re-sizes its workspace (allocates and synchronises once).
 * MAD_EINVAL for an unknown option or value, MAD_EUNSUPPORTED for an option
 * the plan's kind does not have; MIPS plans have none of these options.
 * ------------------------------------------------------------------------- */
enum { MAD_OPT_ACCUM = 0, MAD_OPT_SAMPLER_ORDER = 1, MAD_OPT_ORDER_CHUNK = 2 };
enum { MAD_ACCUM_PAIRS = 0, MAD_ACCUM_HASH = 1 };
int mad_plan_set_option(mad_plan* plan, int option, int64_t value);
int mad_plan_get_option(mad_plan* plan, int option, int64_t* value);

/* One-shot form of the two calls above for dense inputs:
 * create + topk + destroy.  Synchronises `stream` before returning. */
int mad_topk(const float* A, int64_t m, const float* B, int64_t n, int64_t d,
             int64_t t, int64_t s, int64_t t_prime, uint64_t seed,
             mad_pair* out, int64_t* n_out, void* stream);

/* Release a plan and its device memory (synchronises the device first). */
void mad_plan_destroy(mad_plan* plan);

/* ---------------------------------------------------------------------------
 * Plan statistics of the last mad_plan_topk (host outputs, synchronises):
 *   wnorm    ||W||_1 (FP64, the weights w_ki of Alg. 3, summed)
 *   closed   closed three-paths (diamonds) among the s samples
 *   distinct pairs with at least one closed diamond (nnz(X) <= s, Sec. 3.1)
 *   n_pos    pairs with x_ij > 0 (|Omega_s|, Alg. 2)
 *   n_cand   verified candidates (|Omega_t'|)
 * Any pointer may be NULL.
 * ------------------------------------------------------------------------- */
int mad_plan_stats(mad_plan* plan, double* wnorm, int64_t* closed,
                   int64_t* distinct, int64_t* n_pos, int64_t* n_cand);

/* ---------------------------------------------------------------------------
 * Phase durations (milliseconds, host array `ms` of capacity n) of the last
 * mad_plan_refresh / mad_plan_topk of a plan made with MAD_FLAG_TIMING,
 * measured with HIP events recorded on the launch stream:
 *   ms[0] table construction (mad_plan_refresh or creation)
 *   ms[1] sampling kernel (Alg. 3 loop; with the hash form of X it
 *         includes the score table updates)
 *   ms[2] postprocessing (Alg. 2: selections, verification, output)
 *   ms[3] clearing the score table before sampling (hash form)
 *   ms[4] score accumulation from the per-sample pairs (pair form)
 *   ms[5] the sampling kernel alone (ms[1] less the k-order passes; dense
 *         plans)
 * Synchronises on the last event.  MAD_EINVAL without MAD_FLAG_TIMING.
 * ------------------------------------------------------------------------- */
int mad_plan_phase_ms(mad_plan* plan, double* ms, int n);

/* ---------------------------------------------------------------------------
 * mad_bruteforce_topk -- exhaustive t-MAD (Definition 1) on the matrix
 * cores: every pair's a_i . b_j, top t by |c| (ties by (i, j) ascending),
 * the role of the exact baseline of Sec. 5.3.  The m x n product is never
 * stored: a GEMM over every 64th row of A (or 8th / all rows when m is
 * small) gives a threshold, a second GEMM keeps only the pairs whose
 * computed value plus an a-priori error bound reaches it, and those
 * survivors are re-ranked with fp32 dot products (the same arithmetic as
 * the sampled path's verification).
 *   precision  MAD_FP32, MAD_BF16 or MAD_FP8_E4M3: input type of the GEMM
 *              (fp32 accumulation; fp8 with a per-vector power-of-two scale)
 *   t_screen   0: certified mode: the filter adds an a-priori bound on the
 *              GEMM's rounding error, so the result is the exact top t of
 *              the fp32 products for every precision (for fp8 on data with
 *              small |c| relative to ||a|| ||b|| the bound keeps many pairs).
 *              > 0 with MAD_BF16 / MAD_FP8_E4M3: screening mode: the
 *              t_screen pairs with the largest low-precision |c| are
 *              re-ranked in fp32 (not certified; callers report recall).
 *   out, n_out (device) as for mad_plan_topk (x = 0)
 *   stats      (host, optional) phase times and survivor count
 * Synchronises `stream`.  Keeps a process-wide workspace between calls.
 * ------------------------------------------------------------------------- */
typedef struct mad_bf_stats {
  double ms_screen;    /* conversion + threshold GEMM                     */
  double ms_filter;    /* all-pairs GEMM with the bound filter            */
  double ms_rerank;    /* fp32 re-rank and the exact selection            */
  int64_t candidates;  /* survivors of the filter                         */
  float tau;           /* filter threshold                                */
  int64_t row_stride;  /* the threshold GEMM used every row_stride-th row */
  int64_t reranked;    /* pairs re-ranked in fp32                         */
} mad_bf_stats;

int mad_bruteforce_topk(const float* A, int64_t m, const float* B, int64_t n,
                        int64_t d, int precision, int64_t t, int64_t t_screen,
                        mad_pair* out, int64_t* n_out, mad_bf_stats* stats,
                        void* stream);

/* ---------------------------------------------------------------------------
 * mad_bruteforce_topk_csr -- exhaustive t-MAD (Definition 1) for sparse
 * inputs, the exact baseline of Sec. 5.3 whose cost is the number of
 * wedges (pairs of entries that share a coordinate).  The coordinates with
 * the most wedges ("heavy", deg_A(k) deg_B(k) largest) are copied into
 * dense columns and their part of every a_i . b_j goes through the matrix
 * core brute force (certified filter, `precision` as in
 * mad_bruteforce_topk); the wedges of the other coordinates are listed and
 * summed per pair.  A lower bound on the t-th largest |c| (exact values of
 * the heavy part's top candidates) prunes both parts, and the union of
 * their candidates is re-ranked with fp32 sparse dot products: the result
 * is the top t by |c| of the pairs with c != 0 (ties by (i, j) ascending),
 * as for mad_plan_topk, x = 0.
 *   CSR arrays as for mad_plan_create_csr (device; validated, MAD_EINVAL
 *   when malformed or non-finite).  heavy: number of heavy coordinates, 0
 *   to take the fewest (a multiple of 64) that leave at most 2^30 light
 *   wedges; MAD_EUNSUPPORTED when that needs more than 4096.
 *   out, n_out (device) as for mad_plan_topk; stats (host, optional).
 * Memory: dense copies of 4 (m + n) H bytes and about 40 bytes per light
 * wedge.  Synchronises; keeps a process-wide workspace between calls.
 * ------------------------------------------------------------------------- */
typedef struct mad_bf_csr_stats {
  double ms_split;          /* degrees, split, dense copies, light lists   */
  double ms_heavy;          /* brute force of the heavy part, its bound    */
  double ms_light;          /* light wedges summed per pair, pruning       */
  double ms_final;          /* union of the candidates, exact re-rank      */
  int64_t heavy;            /* heavy coordinates                            */
  int64_t wedges;           /* sum over k of deg_A(k) deg_B(k)              */
  int64_t light_wedges;     /* wedges at light coordinates (listed)         */
  int64_t heavy_candidates; /* pairs kept by the heavy part's filter        */
  int64_t light_candidates; /* pairs sharing a light coordinate kept        */
  int64_t candidates;       /* distinct pairs re-ranked                     */
  float tau;                /* the lower bound used for the t-th |c|        */
} mad_bf_csr_stats;

int mad_bruteforce_topk_csr(const int64_t* a_ptr, const int32_t* a_idx,
                            const float* a_val, int64_t m,
                            const int64_t* b_ptr, const int32_t* b_idx,
                            const float* b_val, int64_t n, int64_t d,
                            int precision, int64_t t, int64_t heavy,
                            mad_pair* out, int64_t* n_out,
                            mad_bf_csr_stats* stats, void* stream);

/* ---------------------------------------------------------------------------
 * mad_probe_memory -- measurement kernels for the memory ceilings the
 * sampler works against (used by the benchmark's roofline).  buf (device)
 * holds nwords 64-bit words, nwords a power of two; nops operations at
 * addresses mix64(op index ^ seed) mod nwords:
 *   kind 0 random 8-byte loads        kind 1 random 4-byte loads
 *   kind 2 random 64-bit atomic adds  kind 3 random 64-bit compare-and-swaps
 *   kind 4 compare-and-swap on an aligned word pair followed by an add to
 *          its second word (one insert of a new key into the score table)
 *   kind 5 streaming copy of words [0, nops) to [nwords/2, nwords/2 + nops)
 *          (nops <= nwords/2)
 * Kinds 2-5 modify buf.  Enqueued on `stream`; MAD_EINVAL on bad arguments.
 * ------------------------------------------------------------------------- */
int mad_probe_memory(int kind, void* buf, int64_t nwords, int64_t nops,
                     uint64_t seed, void* stream);

/* ---------------------------------------------------------------------------
 * MIPS (maximum inner product search): Sec. 2 notes that MAD with a single
 * vector on one side is MIPS, and Sec. 6 runs Alg. 3 with Alg. 2 once per
 * query vector with a sample budget s and a dot-product budget t'.
 *
 * mips_plan_create -- preprocessing of the database side of Alg. 3:
 * na_i = ||a_i||_1, v_k, and the alias tables T1[k] (i given k, weight
 * |a_ki| na_i) and T3[i] (k' given i, weight |a_k'i|), shared by every
 * query.  A (device) m x d fp32 row-major, borrowed as by
 * mad_plan_create_dense; 1 <= m < 2^31, 1 <= d <= 4096 (MAD_EUNSUPPORTED
 * above).  Destroy with mad_plan_destroy; mad_plan_refresh rebuilds the
 * tables after A changed.  Synchronises once (input check).
 * ------------------------------------------------------------------------- */
int mips_plan_create(const float* A, int64_t m, int64_t d, uint32_t flags,
                     void* stream, mad_plan** plan);

/* ---------------------------------------------------------------------------
 * mips_topk_batch -- nq queries in one batch.  Query q (row q of Q) gets
 * exactly the result of mad_plan_topk on a plan with B = {q} (n = 1) using
 * s = s_per_query[q], t' = tprime_per_query[q], the same t and seed, and
 * Philox counter word 1 = q: its own stage-0 table (weight |q_k| v_k), its
 * own fixed-point exponent F_q from max|q_k| and s_q, scores keyed by i.
 * A score shares a 64-bit slot with its key, so F_q is the general plan's
 * exponent minus kb, the bit length of m (the scores stay exact).
 *   Q                  (device) nq x d fp32 row-major; 0 <= nq < 2^31
 *   s_per_query        (host) nq budgets, 0 <= s_q < 2^31
 *   tprime_per_query   (host) nq candidate budgets, each >= t
 *   t                  1 <= t <= min(1024, m)
 *   out                (device) nq x t mad_pair; row q holds the top t of
 *                      query q by |c| (ties by i ascending), j = q
 *   n_out              (device) nq int64: pairs written for each query;
 *                      -1 for a query holding NaN or Inf
 * The launches of a batch (per-query exponents and stage-0 tables, the
 * clearing of the score tables, one persistent sampling launch over chunks
 * of every query's samples, one postprocessing launch with a workgroup per
 * query) are captured once into a HIP graph, which later calls with the
 * same Q, out, n_out, seed and budgets replay on `stream`.  A new budget
 * vector re-plans the batch (host work, uploads and allocation: the call
 * then synchronises).  With MAD_FLAG_TIMING the launches run directly,
 * with phase events read by mad_plan_phase_ms.
 * ------------------------------------------------------------------------- */
int mips_topk_batch(mad_plan* plan, const float* Q, int64_t nq,
                    const int64_t* s_per_query, const int64_t* tprime_per_query,
                    int64_t t, uint64_t seed, mad_pair* out, int64_t* n_out,
                    void* stream);

/* Launch shape of the batch (never changes a result): samples per chunk
 * (multiple of 256), samples in flight per thread (1, 2, 4, 8) and
 * workgroups of the persistent sampling launch. */
int mips_get_config(mad_plan* plan, int* chunk, int* unroll, int* grid);
int mips_set_config(mad_plan* plan, int chunk, int unroll, int grid);

/* Score-table slots per possible key of a query (2, 4 or 8; default 2):
 * query q's open-addressing table holds factor * max(min(s_q, m), 512)
 * slots rounded up to a power of two.  A larger table passes fewer taken
 * slots per insert but takes longer to clear and to scan; results never
 * change.  A new factor re-plans the next batch. */
int mips_get_table_factor(mad_plan* plan, int* slots_per_key);
int mips_set_table_factor(mad_plan* plan, int slots_per_key);

/* Autotuner: runs the batch (arguments as mips_topk_batch) under a set of
 * launch shapes and table factors, `reps` timed replays each, keeps the
 * fastest in the plan and reports its time per batch in *best_ms (host,
 * optional).  Results are identical under every shape.  Synchronises.
 * With a choice file (mips_autotune_cache), a batch whose signature (the
 * device's architecture, m, d, nq, the sum and largest of the s_q, the
 * sum of the t'_q, t and the verification precision) is in the file takes
 * the stored choice and its time without any trial; otherwise the tuned
 * choice is appended to the file (MAD_EINVAL when it cannot be written). */
int mips_autotune(mad_plan* plan, const float* Q, int64_t nq,
                  const int64_t* s_per_query, const int64_t* tprime_per_query,
                  int64_t t, uint64_t seed, mad_pair* out, int64_t* n_out,
                  int reps, void* stream, double* best_ms);

/* Text file of the autotuner's choices for this plan (host path, copied;
 * NULL or "" = none): one line per signature, "<signature> | chunk unroll
 * grid slots_per_key ms"; the last line of a signature counts.  Calls that
 * write one file from several processes at once may interleave lines. */
int mips_autotune_cache(mad_plan* plan, const char* path);

/* Statistics of the last batch (synchronises): n_pos[q] = |Omega_s| and
 * n_cand[q] = verified candidates (host arrays of nq, optional), closed
 * diamonds and distinct (query, i) keys over the batch. */
int mips_stats(mad_plan* plan, int64_t* n_pos, int64_t* n_cand,
               int64_t* closed, int64_t* distinct);

/* Score table of query q after the last batch: keys i (device int64) and
 * x_fix (device int64), capacity cap, unordered; *n (host) = count,
 * *F (host) = the query's fixed-point exponent.  Synchronises. */
int mips_debug_scores(mad_plan* plan, int64_t q, int64_t* keys, int64_t* xfix,
                      int64_t cap, int64_t* n, int* F);

/* Thread-local description of the last error (empty string if none). */
const char* mad_last_error(void);

/* ---------------------------------------------------------------------------
 * Parity / debug entry points (not on the hot path).  All synchronise.
 *
 * mad_debug_table: copy one alias table.  which = 0: T0; 1: T1[idx] (over
 * i for coordinate idx); 2: T2[idx] (over j); 3: T3[idx] (over k' for
 * vector idx).  thr, alias (host) receive 2^L words each (capacity cap);
 * entry r gives item r with probability thr/2^31 and alias[r] otherwise
 * (positions; item (host, optional, capacity cap) maps position -> index).
 * *nslots (host) = 2^L.  Returns MAD_EINVAL if cap < 2^L.
 * ------------------------------------------------------------------------- */
int mad_debug_table(mad_plan* plan, int which, int64_t idx, uint32_t* thr,
                    uint32_t* alias, int32_t* item, int64_t cap,
                    int64_t* nslots);

/* FP64 norms: na (host, m), nb (host, d), v (host, d), om (host, d); any
 * may be NULL. */
int mad_debug_norms(mad_plan* plan, double* na, double* nb, double* v,
                    double* om);

/* Per-sample stream of samples l0 .. l0+count-1 (the draws and the score update of Alg. 3):
 * k, i, j, kp (device int32) and inc (device int64: the fixed-point
 * increment, 0 when b_k'j = 0).  F is the fixed-point exponent to use;
 * qid is the query word of the counter (0 for MAD). */
int mad_debug_samples(mad_plan* plan, uint64_t seed, uint64_t qid,
                      int64_t l0, int64_t count, int F, int32_t* k,
                      int32_t* i, int32_t* j, int32_t* kp, int64_t* inc,
                      void* stream);

/* The score accumulation alone, for tests (the pair form of the score update of
 * Alg. 3): over n pairs (keys: device uint64, ~0 = none; vals: device fp32)
 * every key's sum of rne(val * 2^F) as int64, written unordered to
 * out_keys / out_x (device int64, capacity cap); *n_out (host) = number of
 * distinct keys.  The inputs are not modified.  Synchronises;
 * MAD_EOVERFLOW if cap is too small. */
int mad_debug_accumulate(const uint64_t* keys, const float* vals, int64_t n,
                         int F, int64_t* out_keys, int64_t* out_x,
                         int64_t cap, int64_t* n_out, void* stream);

/* ---------------------------------------------------------------------------
 * mad_accumulate_noalloc -- mad_debug_accumulate for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops): the same sums, per key, of rne(vals[e] * 2^F) over the n pairs
 * (keys (device) uint64, ~0 = none; vals (device) fp32), written to
 * out_keys / out_x (device int64, capacity n, unordered); *n_out (device
 * int64) = number of distinct keys.  The inputs are not modified.
 * Allocates nothing and does not synchronise: its workspace is a static
 * device array of 12 MiB that each GPU holds until the process ends, so n
 * is at most 2^18 (MAD_EINVAL above).  Calls that overlap on one GPU share
 * that array and race: serialise them (one stream, or events).  The first
 * call on a device looks up the array's address there.  0 <= F <= 62.
 * ------------------------------------------------------------------------- */
int mad_accumulate_noalloc(const uint64_t* keys, const float* vals, int64_t n,
                           int F, int64_t* out_keys, int64_t* out_x,
                           int64_t* n_out, void* stream);

/* Score table X of the last mad_plan_topk: every pair with a closed
 * diamond, unordered.  keys (device int64, i*n + j), xfix (device int64),
 * capacity cap; *n (host) = number of pairs; *F (host) = fixed-point
 * exponent used.  Returns MAD_EOVERFLOW if cap is too small. */
int mad_debug_scores(mad_plan* plan, int64_t* keys, int64_t* xfix,
                     int64_t cap, int64_t* n, int* F);

/* Candidates Omega_t' of the last mad_plan_topk, unordered: keys, xfix
 * (device int64), c (device fp32), capacity cap; *n (host). */
int mad_debug_candidates(mad_plan* plan, int64_t* keys, int64_t* xfix,
                         float* c, int64_t cap, int64_t* n);

/* Low-precision screen of pairs (measurement of the verification filter of
 * mad_plan_set_verify_precision): for each key i*n + j (device int64),
 * chat = the bf16 / fp8 value c^ of a_i . b_j and margin = its a-priori
 * bound on |c^ - c_fp32| (device fp32 arrays of count).  Needs a dense
 * plan with MAD_BF16 or MAD_FP8_E4M3 verification.  Enqueued on stream. */
int mad_debug_lowp_screen(mad_plan* plan, const int64_t* keys, int64_t count,
                          float* chat, float* margin, void* stream);

/* Fixed-point exponent F the plan uses for s samples (host). */
int mad_fix_exponent(mad_plan* plan, int64_t s, int* F);

#ifdef __cplusplus
}
#endif

#endif /* MAD_H */

/*
 * mad_oracle.c -- plain, slow CPU oracle for diamond sampling.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no code with the GPU library.
 *
 * What it computes (Ballard, Kolda, Pinar, Seshadhri, "Diamond Sampling for
 * Approximate Maximum All-pairs Dot-product (MAD) Search"):
 *   - Alg. 3 (diamond sampling, general inputs): the weights w_ki,
 *     the s draws and the score update;
 *   - Alg. 2 (postprocessing): top-t' of X over {x_ij > 0}, exact dot
 *     products of those candidates, top-t of the result;
 *   - the exhaustive t-MAD answer (Definition 1) by brute force.
 *
 * The paper fixes the distributions but not the arithmetic.  The readings
 * taken here (each one also stated where it is used) are:
 *   R1  vectors are rows of row-major arrays: A is m x d, B is n x d, so
 *       a_ki of the paper is A[i*d + k] (Sec. 2 puts vectors in columns of
 *       d x m matrices; the memory is the same).
 *   R2  (k,i) is drawn in two stages: k with weight nb_k * v_k, then i given
 *       k with weight |a_ki| * na_i, where na_i = ||a_i||_1, nb_k = ||B_k*||_1
 *       and v_k = sum_i |a_ki| na_i.  The product of the two stage
 *       probabilities is exactly w_ki / ||W||_1, the draw of (k, i) in Alg. 3
 *       (Lemma 1's proof factors the same way).
 *   R3  every FP64 sum and prefix sum uses the two-level run order of
 *       prefix_runs() below; products are single IEEE roundings.
 *   R4  each discrete distribution becomes integer quanta q_r that sum to
 *       exactly 2^(L+31) (an integer CDF of the normalised cumulative sums
 *       of Sec. 5.1), then an alias table (Sec. 5.1 names the alias method)
 *       with 2^L slots of capacity 2^31 built by the canonical sweep below.
 *   R5  random numbers: one Philox4x64-10 block per sample l, counter
 *       (l, qid, 0, 0), key (seed, 0); word 0 draws k, word 1 draws i,
 *       word 2 draws j, word 3 draws k'.
 *   R6  the sign factor of the score update is the XOR of the three IEEE sign bits
 *       (the line reads sgn(a_ki b_kj a_k'i); Lemma 2's statement and proof
 *       misprint its subscripts, and its algebra needs the line's form).
 *   R7  scores are exact int64 fixed point: inc = sign * rne(b_k'j * 2^F)
 *       with F = 62 - e_b - ceil(log2 max(s,2)), max|b| < 2^e_b.  Where a
 *       score shares a 64-bit word with a kb-bit key, F is lowered by kb.
 *   R8  ties in both selections of Alg. 2 are broken by (i, j) ascending,
 *       and the final ranking is by |c_ij| (Definition 1 asks for the
 *       largest |a_i . b_j|; Alg. 2 (final selection) prints c_ij).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RUN 128                /* R3: run length of the two-level sum      */
#define CAP_BITS 31            /* R4: alias slot capacity 2^31             */
#define CAP ((uint64_t)1 << CAP_BITS)
#define COIN_MASK (CAP - 1)

/* ------------------------------------------------------------------------
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As
 * Easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplications
 * with the published multipliers and Weyl key increments.
 * ---------------------------------------------------------------------- */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                       uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(0xD2E7470EE14C6C93ULL, c0, &hi0, &lo0);
    mulhilo64(0xCA5A826395121157ULL, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B97F4A7C15ULL;
    k1 += 0xBB67AE8584CAA73BULL;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------
 * R3: inclusive prefix sums of non-negative FP64 weights, in two levels.
 * The sequence is cut into runs of RUN consecutive terms.  Inside a run the
 * terms are added left to right starting from the run's first term; the run
 * offsets are accumulated left to right from zero (E_0 = 0,
 * E_b = E_{b-1} + S_{b-1}); P_r = l_r in the first run and E_b + l_r after.
 * With this order the prefix is non-decreasing and a zero weight repeats
 * the previous prefix exactly (P at the end of run b-1 is E_b).
 * ---------------------------------------------------------------------- */
void orc_prefix(const double *w, int64_t N, double *P) {
  double E = 0.0;
  for (int64_t b0 = 0; b0 < N; b0 += RUN) {
    int64_t b1 = b0 + RUN < N ? b0 + RUN : N;
    double l = w[b0];
    P[b0] = b0 == 0 ? l : E + l;
    for (int64_t r = b0 + 1; r < b1; ++r) {
      l = l + w[r];
      P[r] = b0 == 0 ? l : E + l;
    }
    E = E + l; /* offset of the next run */
  }
}

/* the run length of R3 (for the tests) */
int orc_run_length(void) { return RUN; }

static int ceil_log2(int64_t N) {
  int L = 0;
  while (((int64_t)1 << L) < N) ++L;
  return L;
}

/* ------------------------------------------------------------------------
 * R4: integer quanta.  With L = ceil(log2 N) and K = L + 31, the integer
 * CDF is F_r = floor(2^K * P_r / T) with T = P_{N-1} (the normalised
 * cumulative sums of Sec. 5.1 scaled to integers); q_r = F_r - F_{r-1}.
 * q is padded with zeros to 2^L entries.  Returns 0 (and all-zero q) when
 * the total weight is zero.
 * ---------------------------------------------------------------------- */
int orc_quanta(const double *w, int64_t N, uint64_t *q) {
  int L = ceil_log2(N);
  int64_t Np = (int64_t)1 << L;
  double *P = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  memset(q, 0, sizeof(uint64_t) * (size_t)Np);
  if (N == 0) { free(P); return 0; }
  orc_prefix(w, N, P);
  double T = P[N - 1];
  if (!(T > 0.0)) { free(P); return 0; }
  uint64_t Fprev = 0;
  for (int64_t r = 0; r < N; ++r) {
    double f = floor(ldexp(P[r] / T, L + CAP_BITS));
    uint64_t F = (uint64_t)f;
    q[r] = F - Fprev;
    Fprev = F;
  }
  free(P);
  return 1;
}

/* ------------------------------------------------------------------------
 * R4: alias table from quanta (the alias method of Sec. 5.1), canonical
 * sweep.  Slots hold capacity C = 2^31.  Light slots (q < C) and heavy slots
 * (q >= C) are each visited in index order.  The current heavy slot donates
 * to each light slot in turn (thr = q_light, alias = heavy); when its own
 * residual w drops below C it is closed as a light slot (thr = w, alias =
 * next heavy) and the next heavy slot becomes the donor, starting from
 * q_next - (C - w).  Heavy slots left at the end hold exactly C and are
 * "full": thr = 0, alias = itself.  A draw picks slot u and coin c in
 * [0, C) and returns u if c < thr[u], else alias[u]; item r is then
 * returned with probability q_r / 2^(L+31) exactly.
 * Returns 0 on success, -1 if the quanta do not sum to 2^L * C.
 * ---------------------------------------------------------------------- */
int orc_alias(const uint64_t *q, int L, uint32_t *thr, uint32_t *alias) {
  int64_t Np = (int64_t)1 << L;
  unsigned __int128 sum = 0;
  for (int64_t r = 0; r < Np; ++r) sum += q[r];
  if (sum != (unsigned __int128)Np * CAP) return -1;
  int64_t *light = (int64_t *)malloc(sizeof(int64_t) * (size_t)Np);
  int64_t *heavy = (int64_t *)malloc(sizeof(int64_t) * (size_t)Np);
  int64_t nl = 0, nh = 0;
  for (int64_t r = 0; r < Np; ++r) {
    if (q[r] < CAP) light[nl++] = r; else heavy[nh++] = r;
  }
  int64_t h = 0;
  int64_t j = heavy[0];
  uint64_t w = q[j];
  for (int64_t a = 0; a < nl; ++a) {
    int64_t l = light[a];
    thr[l] = (uint32_t)q[l];
    alias[l] = (uint32_t)j;
    w -= CAP - q[l];
    while (w < CAP) {
      int64_t jn = heavy[++h]; /* exists: the quanta balance */
      thr[j] = (uint32_t)w;
      alias[j] = (uint32_t)jn;
      w = q[jn] - (CAP - w);
      j = jn;
    }
  }
  for (; h < nh; ++h) {
    thr[heavy[h]] = 0;
    alias[heavy[h]] = (uint32_t)heavy[h];
  }
  free(light);
  free(heavy);
  return 0;
}

/* R4/R5: one draw from an alias table with 2^L slots using a 64-bit word:
 * the slot is the top L bits, the coin the low 31 bits. */
int64_t orc_draw(const uint32_t *thr, const uint32_t *alias, int L,
                 uint64_t U) {
  uint64_t slot = L ? (U >> (64 - L)) : 0;
  uint64_t coin = U & COIN_MASK;
  return coin < thr[slot] ? (int64_t)slot : (int64_t)alias[slot];
}

/* ------------------------------------------------------------------------
 * Sampling tables.  A table is a discrete distribution over "positions";
 * item[] maps a position to the index it stands for (NULL: the position is
 * the index).
 * ---------------------------------------------------------------------- */
typedef struct {
  int64_t N;       /* positions with a weight (before padding) */
  int L;           /* 2^L slots */
  int live;        /* total weight > 0 */
  double total;    /* T = P_{N-1} */
  uint32_t *thr, *alias;
  int32_t *item;   /* position -> index, or NULL */
} otable;

static void table_build(otable *t, const double *w, int64_t N,
                        const int32_t *item) {
  t->N = N;
  t->L = ceil_log2(N);
  int64_t Np = (int64_t)1 << t->L;
  uint64_t *q = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)Np);
  double *P = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  if (N > 0) orc_prefix(w, N, P);
  t->total = N > 0 ? P[N - 1] : 0.0;
  free(P);
  t->live = orc_quanta(w, N, q);
  t->thr = (uint32_t *)calloc((size_t)Np, sizeof(uint32_t));
  t->alias = (uint32_t *)calloc((size_t)Np, sizeof(uint32_t));
  if (t->live) orc_alias(q, t->L, t->thr, t->alias);
  free(q);
  t->item = NULL;
  if (item) {
    t->item = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    memcpy(t->item, item, sizeof(int32_t) * (size_t)N);
  }
}

static void table_free(otable *t) {
  free(t->thr);
  free(t->alias);
  free(t->item);
}

static int64_t table_draw(const otable *t, uint64_t U) {
  int64_t p = orc_draw(t->thr, t->alias, t->L, U);
  return t->item ? t->item[p] : p;
}

/* ------------------------------------------------------------------------
 * Inputs.  Dense: A[i*d+k], B[j*d+k] (R1).  Sparse: one sorted list of
 * (coordinate, value) per vector (compressed rows of the vector-major
 * arrays).  The oracle keeps both as the sparse form, a dense input being
 * all coordinates of every vector, zeros included.
 * ---------------------------------------------------------------------- */
typedef struct {
  int64_t rows, d;
  int64_t *ptr;  /* rows + 1 */
  int32_t *idx;  /* coordinate of each entry, ascending within a row */
  float *val;
} ovecs;

static void vecs_from_dense(ovecs *v, const float *X, int64_t rows,
                            int64_t d) {
  v->rows = rows;
  v->d = d;
  v->ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(rows + 1));
  v->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rows * d + 1));
  v->val = (float *)malloc(sizeof(float) * (size_t)(rows * d + 1));
  for (int64_t r = 0; r <= rows; ++r) v->ptr[r] = r * d;
  for (int64_t r = 0; r < rows; ++r)
    for (int64_t k = 0; k < d; ++k) {
      v->idx[r * d + k] = (int32_t)k;
      v->val[r * d + k] = X[r * d + k];
    }
}

static void vecs_from_csr(ovecs *v, const int64_t *ptr, const int32_t *idx,
                          const float *val, int64_t rows, int64_t d) {
  int64_t nnz = ptr[rows];
  v->rows = rows;
  v->d = d;
  v->ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(rows + 1));
  v->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
  v->val = (float *)malloc(sizeof(float) * (size_t)(nnz + 1));
  memcpy(v->ptr, ptr, sizeof(int64_t) * (size_t)(rows + 1));
  memcpy(v->idx, idx, sizeof(int32_t) * (size_t)nnz);
  memcpy(v->val, val, sizeof(float) * (size_t)nnz);
}

static void vecs_free(ovecs *v) {
  free(v->ptr);
  free(v->idx);
  free(v->val);
}

/* value of coordinate k in vector r (0 if absent): binary search */
static float vecs_get(const ovecs *v, int64_t r, int32_t k) {
  int64_t lo = v->ptr[r], hi = v->ptr[r + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (v->idx[mid] < k) lo = mid + 1; else hi = mid;
  }
  return (lo < v->ptr[r + 1] && v->idx[lo] == k) ? v->val[lo] : 0.0f;
}

/* Transposed view: for each coordinate k, the vectors with an entry at k
 * (in ascending vector order, dense inputs included with zeros). */
typedef struct {
  int64_t *ptr; /* d + 1 */
  int32_t *row; /* vector index */
  float *val;
} otrans;

static void trans_build(otrans *t, const ovecs *v) {
  int64_t d = v->d, nnz = v->ptr[v->rows];
  t->ptr = (int64_t *)calloc((size_t)(d + 1), sizeof(int64_t));
  t->row = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
  t->val = (float *)malloc(sizeof(float) * (size_t)(nnz + 1));
  for (int64_t e = 0; e < nnz; ++e) t->ptr[v->idx[e] + 1]++;
  for (int64_t k = 0; k < d; ++k) t->ptr[k + 1] += t->ptr[k];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(d + 1));
  memcpy(fill, t->ptr, sizeof(int64_t) * (size_t)(d + 1));
  for (int64_t r = 0; r < v->rows; ++r)
    for (int64_t e = v->ptr[r]; e < v->ptr[r + 1]; ++e) {
      int64_t p = fill[v->idx[e]]++;
      t->row[p] = (int32_t)r;
      t->val[p] = v->val[e];
    }
  free(fill);
}

static void trans_free(otrans *t) {
  free(t->ptr);
  free(t->row);
  free(t->val);
}

/* ------------------------------------------------------------------------
 * The oracle plan: everything that the weights w_ki of Alg. 3 and the
 * draws need.
 *   na[i]  = ||a_i||_1         total of T3[i]
 *   nb[k]  = ||B_k*||_1        total of T2[k]
 *   v[k]   = sum_i |a_ki| na_i total of T1[k]
 *   om[k]  = nb[k] * v[k]      weights of T0;  ||W||_1 = total of T0
 * ---------------------------------------------------------------------- */
typedef struct orc_plan {
  ovecs A, B;
  otrans At, Bt;
  int64_t m, n, d;
  double *na, *nb, *v, *om;
  otable T0;
  otable *T1, *T2, *T3;
  float bmax;   /* max |b| over all entries */
  int gram;     /* B = A: symmetrise X and drop the diagonal (Sec. 3.2.2) */
  int square;   /* B = A symmetric, C = A^2: two updates per sample
                   (Sec. 3.2.3), then the symmetrisation of gram */
} orc_plan;

static void plan_build_aside(orc_plan *p) {
  int64_t m = p->m, d = p->d;
  p->na = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
  p->T3 = (otable *)calloc((size_t)(m > 0 ? m : 1), sizeof(otable));
  /* T3[i]: k' given i with weight |a_k'i| (the draw of k' in Alg. 3) */
  for (int64_t i = 0; i < m; ++i) {
    int64_t e0 = p->A.ptr[i], N = p->A.ptr[i + 1] - e0;
    double *w = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int64_t e = 0; e < N; ++e) w[e] = fabs((double)p->A.val[e0 + e]);
    table_build(&p->T3[i], w, N, p->A.idx + e0);
    p->na[i] = p->T3[i].total;
    free(w);
  }
  /* T1[k]: i given k with weight |a_ki| * na_i (R2) */
  trans_build(&p->At, &p->A);
  p->v = (double *)calloc((size_t)(d > 0 ? d : 1), sizeof(double));
  p->T1 = (otable *)calloc((size_t)(d > 0 ? d : 1), sizeof(otable));
  for (int64_t k = 0; k < d; ++k) {
    int64_t e0 = p->At.ptr[k], N = p->At.ptr[k + 1] - e0;
    double *w = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int64_t e = 0; e < N; ++e)
      w[e] = fabs((double)p->At.val[e0 + e]) * p->na[p->At.row[e0 + e]];
    table_build(&p->T1[k], w, N, p->At.row + e0);
    p->v[k] = p->T1[k].total;
    free(w);
  }
}

static void plan_build_bside(orc_plan *p) {
  int64_t d = p->d;
  trans_build(&p->Bt, &p->B);
  p->nb = (double *)calloc((size_t)(d > 0 ? d : 1), sizeof(double));
  p->T2 = (otable *)calloc((size_t)(d > 0 ? d : 1), sizeof(otable));
  /* T2[k]: j given k with weight |b_kj| (the draw of j in Alg. 3) */
  for (int64_t k = 0; k < d; ++k) {
    int64_t e0 = p->Bt.ptr[k], N = p->Bt.ptr[k + 1] - e0;
    double *w = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int64_t e = 0; e < N; ++e) w[e] = fabs((double)p->Bt.val[e0 + e]);
    table_build(&p->T2[k], w, N, p->Bt.row + e0);
    p->nb[k] = p->T2[k].total;
    free(w);
  }
  /* T0: k with weight om_k = nb_k * v_k (R2); total = ||W||_1 */
  p->om = (double *)calloc((size_t)(d > 0 ? d : 1), sizeof(double));
  for (int64_t k = 0; k < d; ++k) p->om[k] = p->nb[k] * p->v[k];
  table_build(&p->T0, p->om, d, NULL);
  p->bmax = 0.0f;
  for (int64_t e = 0; e < p->B.ptr[p->B.rows]; ++e) {
    float a = fabsf(p->B.val[e]);
    if (a > p->bmax) p->bmax = a;
  }
}

static void plan_free_bside(orc_plan *p) {
  for (int64_t k = 0; k < p->d; ++k) table_free(&p->T2[k]);
  free(p->T2);
  table_free(&p->T0);
  free(p->nb);
  free(p->om);
  trans_free(&p->Bt);
  vecs_free(&p->B);
}

orc_plan *orc_plan_dense(const float *A, int64_t m, const float *B, int64_t n,
                         int64_t d) {
  orc_plan *p = (orc_plan *)calloc(1, sizeof(orc_plan));
  p->m = m; p->n = n; p->d = d;
  vecs_from_dense(&p->A, A, m, d);
  vecs_from_dense(&p->B, B, n, d);
  plan_build_aside(p);
  plan_build_bside(p);
  return p;
}

orc_plan *orc_plan_csr(const int64_t *a_ptr, const int32_t *a_idx,
                       const float *a_val, int64_t m, const int64_t *b_ptr,
                       const int32_t *b_idx, const float *b_val, int64_t n,
                       int64_t d) {
  orc_plan *p = (orc_plan *)calloc(1, sizeof(orc_plan));
  p->m = m; p->n = n; p->d = d;
  vecs_from_csr(&p->A, a_ptr, a_idx, a_val, m, d);
  vecs_from_csr(&p->B, b_ptr, b_idx, b_val, n, d);
  plan_build_aside(p);
  plan_build_bside(p);
  return p;
}

/* Replace B by a new dense set (used for one query at a time in MIPS,
 * where B is a single vector); the A-side tables are kept. */
void orc_plan_set_dense_b(orc_plan *p, const float *B, int64_t n) {
  plan_free_bside(p);
  p->n = n;
  vecs_from_dense(&p->B, B, n, p->d);
  plan_build_bside(p);
}

void orc_plan_free(orc_plan *p) {
  if (!p) return;
  for (int64_t i = 0; i < p->m; ++i) table_free(&p->T3[i]);
  for (int64_t k = 0; k < p->d; ++k) table_free(&p->T1[k]);
  free(p->T3); free(p->T1);
  free(p->na); free(p->v);
  trans_free(&p->At);
  vecs_free(&p->A);
  plan_free_bside(p);
  free(p);
}

double orc_plan_wnorm(const orc_plan *p) { return p->T0.total; }

void orc_plan_norms(const orc_plan *p, double *na, double *nb, double *v,
                    double *om) {
  if (na) memcpy(na, p->na, sizeof(double) * (size_t)p->m);
  if (nb) memcpy(nb, p->nb, sizeof(double) * (size_t)p->d);
  if (v) memcpy(v, p->v, sizeof(double) * (size_t)p->d);
  if (om) memcpy(om, p->om, sizeof(double) * (size_t)p->d);
}

/* Copy out one table: which = 0 (T0), 1 (T1[idx]), 2 (T2[idx]),
 * 3 (T3[idx]).  Returns the slot count 2^L, or -1 for a bad index; thr,
 * alias, item may be NULL to query the size.  live/total/N are optional. */
int64_t orc_plan_table(const orc_plan *p, int which, int64_t idx,
                       uint32_t *thr, uint32_t *alias, int32_t *item,
                       int64_t *N, int32_t *live, double *total) {
  const otable *t;
  if (which == 0) t = &p->T0;
  else if (which == 1 && idx >= 0 && idx < p->d) t = &p->T1[idx];
  else if (which == 2 && idx >= 0 && idx < p->d) t = &p->T2[idx];
  else if (which == 3 && idx >= 0 && idx < p->m) t = &p->T3[idx];
  else return -1;
  int64_t Np = (int64_t)1 << t->L;
  if (thr) memcpy(thr, t->thr, sizeof(uint32_t) * (size_t)Np);
  if (alias) memcpy(alias, t->alias, sizeof(uint32_t) * (size_t)Np);
  if (item) {
    for (int64_t r = 0; r < t->N; ++r) item[r] = t->item ? t->item[r] : (int32_t)r;
  }
  if (N) *N = t->N;
  if (live) *live = t->live;
  if (total) *total = t->total;
  return Np;
}

/* R7: fixed-point exponent F for s samples. */
int orc_fix_exponent(float bmax, int64_t s) {
  int eb;
  frexpf(bmax, &eb); /* bmax = f * 2^eb, f in [0.5,1): bmax < 2^eb */
  int ls = ceil_log2(s > 2 ? s : 2);
  return 62 - eb - ls;
}

/* The squared variant adds two increments per sample, so its exponent is
 * taken for 2s updates (no int64 sum can overflow). */
int orc_plan_fix_exponent(const orc_plan *p, int64_t s) {
  return orc_fix_exponent(p->bmax, p->square ? 2 * s : s);
}

/* R7 for a score kept beside a kb-bit key in one 64-bit word: 64 - kb bits
 * remain for it, so the exponent is lower by kb and any sum of s
 * increments still lies within 2^(62 - kb). */
int orc_plan_fix_exponent_keyed(const orc_plan *p, int64_t s, int kb) {
  return orc_plan_fix_exponent(p, s) - kb;
}

static int sign_bit(float x) {
  uint32_t u;
  memcpy(&u, &x, sizeof u);
  return (int)(u >> 31);
}

/* ------------------------------------------------------------------------
 * One iteration of the sampling loop of Alg. 3 (its draws and score update) for
 * sample l.  Returns 1 and fills *inc when the three-path closes
 * (b_k'j != 0), else 0.  k, i, j, kp are always filled.
 * ---------------------------------------------------------------------- */
static int one_sample(const orc_plan *p, uint64_t seed, uint64_t qid,
                      uint64_t l, int F, int32_t *k_, int32_t *i_,
                      int32_t *j_, int32_t *kp_, int64_t *inc) {
  uint64_t ctr[4] = {l, qid, 0, 0}, key[2] = {seed, 0}, U[4];
  orc_philox4x64_10(ctr, key, U);
  /* draw of (k, i): with probability w_ki / ||W||_1, in two stages (R2) */
  int64_t k = table_draw(&p->T0, U[0]);
  int64_t i = table_draw(&p->T1[k], U[1]);
  /* draw of j: with probability |b_kj| / ||B_k*||_1 */
  int64_t j = table_draw(&p->T2[k], U[2]);
  /* draw of k': with probability |a_k'i| / ||a_i||_1 */
  int64_t kp = table_draw(&p->T3[i], U[3]);
  *k_ = (int32_t)k; *i_ = (int32_t)i; *j_ = (int32_t)j; *kp_ = (int32_t)kp;
  /* dx: x_ij += sgn(a_ki b_kj a_k'i) b_k'j */
  float bkpj = vecs_get(&p->B, j, (int32_t)kp);
  if (bkpj == 0.0f) { *inc = 0; return 0; }
  float aki = vecs_get(&p->A, i, (int32_t)k);
  float bkj = vecs_get(&p->B, j, (int32_t)k);
  float akpi = vecs_get(&p->A, i, (int32_t)kp);
  int neg = sign_bit(aki) ^ sign_bit(bkj) ^ sign_bit(akpi);
  double scaled = ldexp((double)bkpj, F); /* exact */
  int64_t mag = (int64_t)nearbyint(scaled); /* round half to even */
  *inc = neg ? -mag : mag;
  return 1;
}

/* Per-sample stream for samples l0 .. l0+count-1 (k, i, j, k', inc; inc = 0
 * for a three-path that does not close).  Returns the closed count, or -1
 * when the plan has no weight. */
int64_t orc_plan_samples(const orc_plan *p, uint64_t seed, uint64_t qid,
                         int64_t l0, int64_t count, int F, int32_t *k,
                         int32_t *i, int32_t *j, int32_t *kp, int64_t *inc) {
  if (!p->T0.live) return -1;
  int64_t closed = 0;
  for (int64_t e = 0; e < count; ++e)
    closed += one_sample(p, seed, qid, (uint64_t)(l0 + e), F, &k[e], &i[e],
                         &j[e], &kp[e], &inc[e]);
  return closed;
}

/* ------------------------------------------------------------------------
 * X after s samples: the sorted list of (key = i*n + j, x_fix) with at
 * least one closed diamond.  Built by collecting every closed sample and
 * sorting by key, then summing equal keys.
 * ---------------------------------------------------------------------- */
typedef struct { int64_t key, inc; } kv;

static int cmp_kv_key(const void *a, const void *b) {
  int64_t x = ((const kv *)a)->key, y = ((const kv *)b)->key;
  return (x > y) - (x < y);
}

/* Sec. 3.2.2, equal inputs: X <- (X + X^T) / 2 before Alg. 2.  Kept exact as
 * the integer sum x_ij + x_ji (twice the symmetric entry) under the key of
 * the pair with i < j; the diagonal (a vector paired with itself) is
 * dropped, as in the paper's A^T A experiments.  X is sorted by key; the
 * result is sorted by key too. */
static int64_t find_key(const kv *X, int64_t nd, int64_t key) {
  int64_t lo = 0, hi = nd;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (X[mid].key < key) lo = mid + 1; else hi = mid;
  }
  return (lo < nd && X[lo].key == key) ? lo : -1;
}

static int64_t symmetrise(kv *X, int64_t nd, int64_t n) {
  kv *Y = (kv *)malloc(sizeof(kv) * (size_t)(nd > 0 ? nd : 1));
  int64_t ny = 0;
  for (int64_t e = 0; e < nd; ++e) {
    int64_t i = X[e].key / n, j = X[e].key % n;
    if (i == j) continue;
    int64_t t = find_key(X, nd, j * n + i);
    if (i < j) {
      Y[ny].key = X[e].key;
      Y[ny].inc = X[e].inc + (t >= 0 ? X[t].inc : 0);
      ++ny;
    } else if (t < 0) { /* only (i, j) with i > j was sampled */
      Y[ny].key = j * n + i;
      Y[ny].inc = X[e].inc;
      ++ny;
    }
  }
  qsort(Y, (size_t)ny, sizeof(kv), cmp_kv_key);
  memcpy(X, Y, sizeof(kv) * (size_t)ny);
  free(Y);
  return ny;
}

void orc_plan_set_gram(orc_plan *p, int gram) { p->gram = gram; }

/* Sec. 3.2.3, equal symmetric inputs (C = A^2, B = A, A symmetric, m = d):
 * every closed sample updates x_ij and x_kk' by half of its increment each,
 * then X is symmetrised as in the Gram case.  Kept exact by adding the full
 * increment to both keys: the stored score of a pair i < j is then
 * 2 (x_ij + x_ji), four times the symmetrised entry, which orders the pairs
 * the same way. */
void orc_plan_set_square(orc_plan *p, int square) {
  p->square = square;
  if (square) p->gram = 1;
}

static int64_t build_scores(const orc_plan *p, uint64_t seed, uint64_t qid,
                            int64_t s, int F, kv **out, int64_t *closed_out) {
  const int64_t per = p->square ? 2 : 1;
  kv *all = (kv *)malloc(sizeof(kv) * (size_t)(s > 0 ? per * s : 1));
  int64_t nc = 0, nkv = 0;
  if (p->T0.live) {
    for (int64_t l = 0; l < s; ++l) {
      int32_t k, i, j, kp;
      int64_t inc;
      if (one_sample(p, seed, qid, (uint64_t)l, F, &k, &i, &j, &kp, &inc)) {
        all[nkv].key = (int64_t)i * p->n + j;
        all[nkv].inc = inc;
        ++nkv;
        if (p->square) { /* the second update, of x_kk' */
          all[nkv].key = (int64_t)k * p->n + kp;
          all[nkv].inc = inc;
          ++nkv;
        }
        ++nc;
      }
    }
  }
  qsort(all, (size_t)nkv, sizeof(kv), cmp_kv_key);
  int64_t nd = 0;
  for (int64_t e = 0; e < nkv; ++e) {
    if (nd > 0 && all[nd - 1].key == all[e].key) all[nd - 1].inc += all[e].inc;
    else all[nd++] = all[e];
  }
  if (p->gram) nd = symmetrise(all, nd, p->n);
  *out = all;
  if (closed_out) *closed_out = nc;
  return nd;
}

int64_t orc_plan_scores(const orc_plan *p, uint64_t seed, uint64_t qid,
                        int64_t s, int F, int64_t *keys, int64_t *xfix,
                        int64_t cap, int64_t *closed) {
  kv *X;
  int64_t nd = build_scores(p, seed, qid, s, F, &X, closed);
  for (int64_t e = 0; e < nd && e < cap; ++e) {
    keys[e] = X[e].key;
    xfix[e] = X[e].inc;
  }
  free(X);
  return nd;
}

/* ------------------------------------------------------------------------
 * Alg. 2 postprocessing.
 * ---------------------------------------------------------------------- */
typedef struct { int64_t key; int64_t x; double c; } cand;

/* candidate selection order: x descending, then key (i, j) ascending (R8) */
static int cmp_post1(const void *a, const void *b) {
  const cand *u = (const cand *)a, *v = (const cand *)b;
  if (u->x != v->x) return u->x > v->x ? -1 : 1;
  return (u->key > v->key) - (u->key < v->key);
}

/* final selection order: |c| descending, then key ascending (R8) */
static int cmp_post3(const void *a, const void *b) {
  const cand *u = (const cand *)a, *v = (const cand *)b;
  double x = fabs(u->c), y = fabs(v->c);
  if (x != y) return x > y ? -1 : 1;
  return (u->key > v->key) - (u->key < v->key);
}

/* c_ij = a_i . b_j in FP64, coordinates in ascending order (the fp32
 * products are exact in FP64; the sum rounds). */
static double exact_dot(const orc_plan *p, int64_t i, int64_t j) {
  const ovecs *A = &p->A, *B = &p->B;
  int64_t ea = A->ptr[i], ea1 = A->ptr[i + 1];
  int64_t eb = B->ptr[j], eb1 = B->ptr[j + 1];
  double c = 0.0;
  while (ea < ea1 && eb < eb1) {
    if (A->idx[ea] < B->idx[eb]) ++ea;
    else if (A->idx[ea] > B->idx[eb]) ++eb;
    else {
      c += (double)A->val[ea] * (double)B->val[eb];
      ++ea; ++eb;
    }
  }
  return c;
}

/* Alg. 2 on a given score matrix X (nd entries (key, x_fix), any order):
 * Omega_s = {x > 0}, its top t' by (x desc, key asc), their exact dot
 * products, and the top t by |c|.  Outputs as for orc_plan_topk.  Returns
 * |Omega_t|. */
int64_t orc_plan_post(const orc_plan *p, const int64_t *keys,
                      const int64_t *xfix, int64_t nd, int64_t t_prime,
                      int64_t t, int64_t *tp_key, int64_t *tp_x, double *tp_c,
                      int64_t *n_tp, int64_t *t_key, int64_t *t_x, double *t_c,
                      int64_t *n_pos) {
  cand *c = (cand *)malloc(sizeof(cand) * (size_t)(nd > 0 ? nd : 1));
  int64_t np = 0;
  for (int64_t e = 0; e < nd; ++e)
    if (xfix[e] > 0) { /* Omega_s = {x_ij > 0} */
      c[np].key = keys[e];
      c[np].x = xfix[e];
      c[np].c = 0.0;
      ++np;
    }
  if (n_pos) *n_pos = np;
  /* candidate selection: top-t' of X */
  qsort(c, (size_t)np, sizeof(cand), cmp_post1);
  int64_t ntp = np < t_prime ? np : t_prime;
  /* verification: exact dot products of the candidates */
  for (int64_t e = 0; e < ntp; ++e)
    c[e].c = exact_dot(p, c[e].key / p->n, c[e].key % p->n);
  for (int64_t e = 0; e < ntp; ++e) {
    if (tp_key) tp_key[e] = c[e].key;
    if (tp_x) tp_x[e] = c[e].x;
    if (tp_c) tp_c[e] = c[e].c;
  }
  if (n_tp) *n_tp = ntp;
  /* final selection: top-t of the candidates by |c| */
  qsort(c, (size_t)ntp, sizeof(cand), cmp_post3);
  int64_t nt = ntp < t ? ntp : t;
  for (int64_t e = 0; e < nt; ++e) {
    if (t_key) t_key[e] = c[e].key;
    if (t_x) t_x[e] = c[e].x;
    if (t_c) t_c[e] = c[e].c;
  }
  free(c);
  return nt;
}

/* Full Alg. 3 with Alg. 2 for one (B, qid).  Outputs Omega_{t'} in
 * candidate selection order (tp_* arrays, cap t_prime) and Omega_t in final
 * selection order (t_* arrays, cap t).  Returns |Omega_t|; *n_tp gets
 * |Omega_{t'}|, *n_pos |Omega_s|, *closed the number of closed three-paths. */
int64_t orc_plan_topk(const orc_plan *p, uint64_t seed, uint64_t qid,
                      int64_t s, int64_t t_prime, int64_t t, int F,
                      int64_t *tp_key, int64_t *tp_x, double *tp_c,
                      int64_t *n_tp, int64_t *t_key, int64_t *t_x,
                      double *t_c, int64_t *n_pos, int64_t *closed) {
  kv *X;
  int64_t nd = build_scores(p, seed, qid, s, F, &X, closed);
  int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nd > 0 ? nd : 1));
  int64_t *xfix = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nd > 0 ? nd : 1));
  for (int64_t e = 0; e < nd; ++e) {
    keys[e] = X[e].key;
    xfix[e] = X[e].inc;
  }
  free(X);
  int64_t nt = orc_plan_post(p, keys, xfix, nd, t_prime, t, tp_key, tp_x,
                             tp_c, n_tp, t_key, t_x, t_c, n_pos);
  free(keys);
  free(xfix);
  return nt;
}

/* ------------------------------------------------------------------------
 * Exhaustive t-MAD (Definition 1): every pair's FP64 dot product, top-t by
 * |c| descending then key ascending, kept in a plain sorted array.
 * ---------------------------------------------------------------------- */
int64_t orc_bruteforce_dense(const float *A, int64_t m, const float *B,
                             int64_t n, int64_t d, int64_t t, int64_t *keys,
                             double *cs) {
  int64_t cnt = 0;
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double c = 0.0;
      for (int64_t k = 0; k < d; ++k)
        c += (double)A[i * d + k] * (double)B[j * d + k];
      int64_t key = i * n + j;
      /* insertion into the sorted top list */
      int64_t pos = cnt;
      while (pos > 0) {
        double y = fabs(cs[pos - 1]);
        int before = fabs(c) > y || (fabs(c) == y && key < keys[pos - 1]);
        if (!before) break;
        --pos;
      }
      if (pos >= t) continue;
      int64_t last = cnt < t ? cnt : t - 1;
      for (int64_t e = last; e > pos; --e) {
        keys[e] = keys[e - 1];
        cs[e] = cs[e - 1];
      }
      keys[pos] = key;
      cs[pos] = c;
      if (cnt < t) ++cnt;
    }
  return cnt;
}

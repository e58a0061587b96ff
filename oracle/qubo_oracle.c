/*
 * qubo_oracle.c -- CPU oracle for exhaustive dense-QUBO minimisation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU solver; it is the plain, slow,
 * obviously correct definition the GPU results are checked against.
 *
 * Conventions (paper, Sec. II-B, Fig. "complete state space matrix"):
 *   - a state is a row of the lexicographically ordered matrix U_N, whose
 *     column 0 is the most significant bit: x_i = (index >> (n-1-i)) & 1;
 *   - the objective is the QUBO energy of the Introduction,
 *         E(x) = sum over ALL i, j of Q_ij x_i x_j,
 *     so an upper-triangular Q (Sec. II-A) is just the special case whose
 *     lower triangle is zero;
 *   - the answer is the lexicographic minimum of (E, index): the minimum
 *     energy and, among states that reach it, the lowest index.
 *     Top-k returns the k lexicographically smallest (E, index) pairs.
 *
 * Arithmetic: int32 input is accumulated exactly in int64; fp32 input is
 * converted exactly to double and accumulated in double (round-to-nearest),
 * i ascending then j ascending over the set bits.
 *
 * O1 (oracle_solve_*): direct evaluation of E(x) for every state of an index
 *   range -- the naive O(N^2 2^N) brute force of Sec. I-D.
 * O2 (oracle_gray_*): the textbook O(N 2^N) Gray-code brute force of
 *   Sec. I-D: walk all states in reflected Gray order, updating E by the
 *   single-flip identity E(x ^ e_k) - E(x) = (1 - 2 x_k) f_k(x) with the
 *   local field f_k(x) = Q_kk + sum_{j != k} (Q_kj + Q_jk) x_j, and updating
 *   every field after each flip.  Used as a cross-check of O1 and for n too
 *   large for O1.
 *
 * Parallelism: contiguous shards of the index (O1) or Gray-index (O2) range,
 * one per thread, reduced lexicographically at the end.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORACLE_MAX_N 64
#define ORACLE_MAX_K 4096

/* ------------------------------------------------------------------ */
/* energy of one state, straight from the definition                    */
/* ------------------------------------------------------------------ */

static int64_t energy_i(int n, const int32_t *Q, uint64_t index)
{
    int set[ORACLE_MAX_N];
    int c = 0;
    for (int i = 0; i < n; i++)
        if ((index >> (n - 1 - i)) & 1u) set[c++] = i;
    int64_t E = 0;
    for (int a = 0; a < c; a++)
        for (int b = 0; b < c; b++)
            E += (int64_t)Q[(size_t)set[a] * n + set[b]];
    return E;
}

static double energy_f(int n, const float *Q, uint64_t index)
{
    int set[ORACLE_MAX_N];
    int c = 0;
    for (int i = 0; i < n; i++)
        if ((index >> (n - 1 - i)) & 1u) set[c++] = i;
    double E = 0.0;
    for (int a = 0; a < c; a++)
        for (int b = 0; b < c; b++)
            E += (double)Q[(size_t)set[a] * n + set[b]];
    return E;
}

int oracle_energy_i(int n, const int32_t *Q, uint64_t index, int64_t *E)
{
    if (n < 1 || n > ORACLE_MAX_N || !Q || !E) return -1;
    *E = energy_i(n, Q, index);
    return 0;
}

int oracle_energy_f(int n, const float *Q, uint64_t index, double *E)
{
    if (n < 1 || n > ORACLE_MAX_N || !Q || !E) return -1;
    *E = energy_f(n, Q, index);
    return 0;
}

/* ------------------------------------------------------------------ */
/* top-k list of (E, index), kept sorted ascending lexicographically    */
/* ------------------------------------------------------------------ */

typedef struct {
    double e;   /* energy (int64 values are exact in the int path's own list) */
    int64_t ei;
    uint64_t idx;
} entry_t;

/* lexicographic (E, index) order; is_int selects which energy field counts */
static int entry_less(const entry_t *a, const entry_t *b, int is_int)
{
    if (is_int) {
        if (a->ei != b->ei) return a->ei < b->ei;
    } else {
        if (a->e != b->e) return a->e < b->e;
    }
    return a->idx < b->idx;
}

typedef struct {
    entry_t *v;
    int len, k, is_int;
} topk_t;

static void topk_offer(topk_t *t, const entry_t *c)
{
    if (t->len == t->k && !entry_less(c, &t->v[t->len - 1], t->is_int)) return;
    int pos = (t->len < t->k) ? t->len++ : t->len - 1;
    while (pos > 0 && entry_less(c, &t->v[pos - 1], t->is_int)) {
        t->v[pos] = t->v[pos - 1];
        pos--;
    }
    t->v[pos] = *c;
}

static int resolve_threads(int threads, uint64_t work)
{
    if (threads <= 0) {
        long p = sysconf(_SC_NPROCESSORS_ONLN);
        threads = (p > 0) ? (int)p : 1;
    }
    if (threads > 256) threads = 256;
    if ((uint64_t)threads > work) threads = (int)(work ? work : 1);
    return threads;
}

/* ------------------------------------------------------------------ */
/* O1: direct evaluation over an index range                            */
/* ------------------------------------------------------------------ */

typedef struct {
    int n, is_int;
    const void *Q;
    uint64_t first, count;
    topk_t top;
} o1_job_t;

static void *o1_worker(void *arg)
{
    o1_job_t *j = (o1_job_t *)arg;
    for (uint64_t r = j->first; r < j->first + j->count; r++) {
        entry_t c;
        c.idx = r;
        if (j->is_int) {
            c.ei = energy_i(j->n, (const int32_t *)j->Q, r);
            c.e = (double)c.ei;
        } else {
            c.e = energy_f(j->n, (const float *)j->Q, r);
            c.ei = 0;
        }
        topk_offer(&j->top, &c);
    }
    return NULL;
}

static int o1_solve(int n, const void *Q, int is_int, uint64_t first, uint64_t count,
                    int k, int threads, int64_t *Ei, double *Ef, uint64_t *idx)
{
    if (n < 1 || n > ORACLE_MAX_N || !Q || !idx || k < 1 || k > ORACLE_MAX_K) return -1;
    uint64_t total = (n == 64) ? 0 : (1ull << n);
    if (n < 64 && (first > total || count > total - first)) return -1;
    if (count == 0) return -1;
    int T = resolve_threads(threads, count);
    o1_job_t *jobs = (o1_job_t *)calloc((size_t)T, sizeof(o1_job_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    if (!jobs || !tid) { free(jobs); free(tid); return -2; }
    uint64_t per = count / (uint64_t)T, rem = count % (uint64_t)T, at = first;
    int rc = 0;
    for (int t = 0; t < T; t++) {
        jobs[t].n = n;
        jobs[t].is_int = is_int;
        jobs[t].Q = Q;
        jobs[t].first = at;
        jobs[t].count = per + ((uint64_t)t < rem ? 1 : 0);
        at += jobs[t].count;
        jobs[t].top.k = k;
        jobs[t].top.is_int = is_int;
        jobs[t].top.v = (entry_t *)malloc((size_t)k * sizeof(entry_t));
        if (!jobs[t].top.v) rc = -2;
    }
    if (rc == 0) {
        for (int t = 0; t < T; t++) pthread_create(&tid[t], NULL, o1_worker, &jobs[t]);
        for (int t = 0; t < T; t++) pthread_join(tid[t], NULL);
        topk_t all = {0};
        all.k = k;
        all.is_int = is_int;
        all.v = (entry_t *)malloc((size_t)k * sizeof(entry_t));
        if (!all.v) rc = -2;
        else {
            for (int t = 0; t < T; t++)
                for (int q = 0; q < jobs[t].top.len; q++) topk_offer(&all, &jobs[t].top.v[q]);
            for (int q = 0; q < k; q++) {
                int have = q < all.len;
                idx[q] = have ? all.v[q].idx : UINT64_MAX;
                if (Ei) Ei[q] = have ? all.v[q].ei : INT64_MAX;
                if (Ef) Ef[q] = have ? all.v[q].e : 0.0;
            }
            free(all.v);
        }
    }
    for (int t = 0; t < T; t++) free(jobs[t].top.v);
    free(jobs);
    free(tid);
    return rc;
}

/* k smallest (E, index) over indices [first, first + count); entries past the
 * number of states get index UINT64_MAX. */
int oracle_solve_i(int n, const int32_t *Q, uint64_t first, uint64_t count, int k,
                   int threads, int64_t *E, uint64_t *idx)
{
    if (!E) return -1;
    return o1_solve(n, Q, 1, first, count, k, threads, E, NULL, idx);
}

int oracle_solve_f(int n, const float *Q, uint64_t first, uint64_t count, int k,
                   int threads, double *E, uint64_t *idx)
{
    if (!E) return -1;
    return o1_solve(n, Q, 0, first, count, k, threads, NULL, E, idx);
}

/* ------------------------------------------------------------------ */
/* O2: local-field Gray-code walk over a range of Gray indices          */
/* ------------------------------------------------------------------ */

/* The coupling of variables v and k in the single-flip identity is
 * S_kv = Q_kv + Q_vk for v != k.  O2 stores it row by row, S[k][0..np),
 * with S_kk = 0 and zero padding up to np (a multiple of 8), so that the
 * field update after a flip of k reads one contiguous row.  Adding S_kk = 0
 * to f_k leaves it unchanged, as it must be (f_k does not depend on x_k). */
#define O2_PAD 8

typedef struct {
    int n, np, is_int;
    const void *Q;
    const int64_t *Si;       /* np x np int64 coupling rows (int input) */
    const double *Sf;        /* np x np double coupling rows (fp32 input) */
    uint64_t i0, i1;         /* Gray-index range [i0, i1) */
    int64_t bestEi;
    double bestEf;
    uint64_t bestIdx;
    int have;
} o2_job_t;

/* One walk over the job's Gray-index range, for coupling rows of length np. */
static inline __attribute__((always_inline)) void o2_walk_i_np(o2_job_t *j, const int np)
{
    const int n = j->n;
    const int32_t *Q = (const int32_t *)j->Q;
    int64_t f[ORACLE_MAX_N];
    int x[ORACLE_MAX_N];
    uint64_t row = j->i0 ^ (j->i0 >> 1);  /* reflected Gray code of i0 */
    for (int v = 0; v < n; v++) x[v] = (int)((row >> (n - 1 - v)) & 1u);
    for (int v = n; v < np; v++) f[v] = 0;
    int64_t E = energy_i(n, Q, row);
    for (int k = 0; k < n; k++) {         /* f_k = Q_kk + sum_{v != k} S_kv x_v */
        int64_t s = Q[(size_t)k * n + k];
        for (int v = 0; v < n; v++)
            if (x[v]) s += j->Si[(size_t)k * np + v];
        f[k] = s;
    }
    j->have = 0;
    for (uint64_t i = j->i0;; i++) {
        if (!j->have || E < j->bestEi || (E == j->bestEi && row < j->bestIdx)) {
            j->have = 1;
            j->bestEi = E;
            j->bestIdx = row;
        }
        if (i + 1 >= j->i1) break;
        int t = __builtin_ctzll(i + 1);      /* Gray level that flips */
        int k = n - 1 - t;                   /* vector position, MSB-left */
        const int64_t *S = j->Si + (size_t)k * np;
        row ^= 1ull << t;
        if (x[k]) {                          /* x_k goes 1 -> 0: delta = -1 */
            E -= f[k];
            for (int v = 0; v < np; v++) f[v] -= S[v];
        } else {                             /* x_k goes 0 -> 1: delta = +1 */
            E += f[k];
            for (int v = 0; v < np; v++) f[v] += S[v];
        }
        x[k] ^= 1;
    }
}

static inline __attribute__((always_inline)) void o2_walk_f_np(o2_job_t *j, const int np)
{
    const int n = j->n;
    const float *Q = (const float *)j->Q;
    double f[ORACLE_MAX_N];
    int x[ORACLE_MAX_N];
    uint64_t row = j->i0 ^ (j->i0 >> 1);
    for (int v = 0; v < n; v++) x[v] = (int)((row >> (n - 1 - v)) & 1u);
    for (int v = n; v < np; v++) f[v] = 0.0;
    double E = energy_f(n, Q, row);
    for (int k = 0; k < n; k++) {
        double s = Q[(size_t)k * n + k];
        for (int v = 0; v < n; v++)
            if (x[v]) s += j->Sf[(size_t)k * np + v];
        f[k] = s;
    }
    j->have = 0;
    for (uint64_t i = j->i0;; i++) {
        if (!j->have || E < j->bestEf || (E == j->bestEf && row < j->bestIdx)) {
            j->have = 1;
            j->bestEf = E;
            j->bestIdx = row;
        }
        if (i + 1 >= j->i1) break;
        int t = __builtin_ctzll(i + 1);
        int k = n - 1 - t;
        const double *S = j->Sf + (size_t)k * np;
        row ^= 1ull << t;
        if (x[k]) {
            E -= f[k];
            for (int v = 0; v < np; v++) f[v] -= S[v];
        } else {
            E += f[k];
            for (int v = 0; v < np; v++) f[v] += S[v];
        }
        x[k] ^= 1;
    }
}

/* The row length np is passed as a constant (one copy of the walk per
 * multiple of 8), so the field update compiles to straight-line vector code. */
#define O2_DISPATCH(body, j)                                                    \
    switch ((j)->np) {                                                          \
    case 8: body(j, 8); break;   case 16: body(j, 16); break;                   \
    case 24: body(j, 24); break; case 32: body(j, 32); break;                   \
    case 40: body(j, 40); break; case 48: body(j, 48); break;                   \
    case 56: body(j, 56); break; default: body(j, 64); break;                   \
    }

/* The walk proper, compiled for several instruction sets; the loader picks
 * the widest one the host supports (results do not depend on the choice:
 * every step is exact integer arithmetic or the same double additions).
 * Sanitizer builds define ORACLE_NO_TARGET_CLONES: the loader resolves the
 * clones (ifunc) before a sanitizer runtime has started. */
#ifdef ORACLE_NO_TARGET_CLONES
#define O2_CLONES
#else
#define O2_CLONES __attribute__((target_clones("avx512f", "avx2", "default")))
#endif

O2_CLONES
static void o2_walk_i(o2_job_t *j)
{
    O2_DISPATCH(o2_walk_i_np, j)
}

O2_CLONES
static void o2_walk_f(o2_job_t *j)
{
    O2_DISPATCH(o2_walk_f_np, j)
}

static void *o2_worker(void *arg)
{
    o2_job_t *j = (o2_job_t *)arg;
    if (j->is_int) o2_walk_i(j);
    else o2_walk_f(j);
    return NULL;
}

/* best (E, index) over the Gray indices [i0, i1), i.e. over the states
 * g(i) = i ^ (i >> 1) for i0 <= i < i1 */
static int o2_solve(int n, const void *Q, int is_int, uint64_t i0, uint64_t i1, int threads,
                    int64_t *Ei, double *Ef, uint64_t *idx)
{
    if (n < 1 || n > 62 || !Q || !idx) return -1;
    uint64_t total = 1ull << n;
    if (i0 >= i1 || i1 > total) return -1;
    int T = resolve_threads(threads, i1 - i0);
    int np = (n + O2_PAD - 1) / O2_PAD * O2_PAD;
    int64_t *Si = NULL;
    double *Sf = NULL;
    if (is_int) Si = (int64_t *)calloc((size_t)np * np, sizeof(int64_t));
    else Sf = (double *)calloc((size_t)np * np, sizeof(double));
    o2_job_t *jobs = (o2_job_t *)calloc((size_t)T, sizeof(o2_job_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    if (!jobs || !tid || (!Si && !Sf)) { free(jobs); free(tid); free(Si); free(Sf); return -2; }
    for (int k = 0; k < n; k++)
        for (int v = 0; v < n; v++) {
            if (v == k) continue;
            if (is_int)
                Si[(size_t)k * np + v] = (int64_t)((const int32_t *)Q)[(size_t)k * n + v] +
                                         ((const int32_t *)Q)[(size_t)v * n + k];
            else
                Sf[(size_t)k * np + v] = (double)((const float *)Q)[(size_t)k * n + v] +
                                         (double)((const float *)Q)[(size_t)v * n + k];
        }
    uint64_t count = i1 - i0, per = count / (uint64_t)T, rem = count % (uint64_t)T, at = i0;
    for (int t = 0; t < T; t++) {
        jobs[t].n = n;
        jobs[t].np = np;
        jobs[t].is_int = is_int;
        jobs[t].Q = Q;
        jobs[t].Si = Si;
        jobs[t].Sf = Sf;
        jobs[t].i0 = at;
        at += per + ((uint64_t)t < rem ? 1 : 0);
        jobs[t].i1 = at;
        pthread_create(&tid[t], NULL, o2_worker, &jobs[t]);
    }
    for (int t = 0; t < T; t++) pthread_join(tid[t], NULL);
    int b = 0;
    for (int t = 1; t < T; t++) {
        int better;
        if (is_int)
            better = jobs[t].bestEi < jobs[b].bestEi ||
                     (jobs[t].bestEi == jobs[b].bestEi && jobs[t].bestIdx < jobs[b].bestIdx);
        else
            better = jobs[t].bestEf < jobs[b].bestEf ||
                     (jobs[t].bestEf == jobs[b].bestEf && jobs[t].bestIdx < jobs[b].bestIdx);
        if (better) b = t;
    }
    *idx = jobs[b].bestIdx;
    if (Ei) *Ei = jobs[b].bestEi;
    if (Ef) *Ef = jobs[b].bestEf;
    free(jobs);
    free(tid);
    free(Si);
    free(Sf);
    return 0;
}

int oracle_gray_i(int n, const int32_t *Q, int threads, int64_t *E, uint64_t *idx)
{
    if (!E || n < 1 || n > 62) return -1;
    return o2_solve(n, Q, 1, 0, 1ull << n, threads, E, NULL, idx);
}

int oracle_gray_f(int n, const float *Q, int threads, double *E, uint64_t *idx)
{
    if (!E || n < 1 || n > 62) return -1;
    return o2_solve(n, Q, 0, 0, 1ull << n, threads, NULL, E, idx);
}

/* best (E, index) over the states of Gray indices [i0, i1): a shard of the
 * whole walk, so that long walks can be split and resumed */
int oracle_gray_range_i(int n, const int32_t *Q, uint64_t i0, uint64_t i1, int threads,
                        int64_t *E, uint64_t *idx)
{
    if (!E) return -1;
    return o2_solve(n, Q, 1, i0, i1, threads, E, NULL, idx);
}

int oracle_gray_range_f(int n, const float *Q, uint64_t i0, uint64_t i1, int threads,
                        double *E, uint64_t *idx)
{
    if (!E) return -1;
    return o2_solve(n, Q, 0, i0, i1, threads, NULL, E, idx);
}

/* number of worker threads a call with threads <= 0 uses */
int oracle_default_threads(void)
{
    return resolve_threads(0, UINT64_MAX);
}

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
/* O2: local-field Gray-code walk over all 2^n states                   */
/* ------------------------------------------------------------------ */

typedef struct {
    int n, is_int;
    const void *Q;
    uint64_t i0, i1;         /* Gray-index range [i0, i1) */
    int64_t bestEi;
    double bestEf;
    uint64_t bestIdx;
    int have;
} o2_job_t;

static void *o2_worker(void *arg)
{
    o2_job_t *j = (o2_job_t *)arg;
    const int n = j->n;
    int x[ORACLE_MAX_N];
    uint64_t row = j->i0 ^ (j->i0 >> 1);  /* reflected Gray code of i0 */
    for (int v = 0; v < n; v++) x[v] = (int)((row >> (n - 1 - v)) & 1u);
    j->have = 0;
    if (j->is_int) {
        const int32_t *Q = (const int32_t *)j->Q;
        int64_t f[ORACLE_MAX_N];
        int64_t E = energy_i(n, Q, row);
        for (int k = 0; k < n; k++) {
            int64_t s = Q[(size_t)k * n + k];
            for (int v = 0; v < n; v++)
                if (v != k && x[v]) s += (int64_t)Q[(size_t)k * n + v] + Q[(size_t)v * n + k];
            f[k] = s;
        }
        for (uint64_t i = j->i0;; i++) {
            if (!j->have || E < j->bestEi || (E == j->bestEi && row < j->bestIdx)) {
                j->have = 1;
                j->bestEi = E;
                j->bestIdx = row;
            }
            if (i + 1 >= j->i1) break;
            int t = __builtin_ctzll(i + 1);      /* Gray level that flips */
            int k = n - 1 - t;                   /* vector position, MSB-left */
            int d = x[k] ? -1 : 1;               /* +1 when x_k goes 0 -> 1 */
            E += d * f[k];
            x[k] ^= 1;
            row ^= 1ull << t;
            for (int v = 0; v < n; v++)
                if (v != k) f[v] += d * ((int64_t)Q[(size_t)v * n + k] + Q[(size_t)k * n + v]);
        }
    } else {
        const float *Q = (const float *)j->Q;
        double f[ORACLE_MAX_N];
        double E = energy_f(n, Q, row);
        for (int k = 0; k < n; k++) {
            double s = Q[(size_t)k * n + k];
            for (int v = 0; v < n; v++)
                if (v != k && x[v]) s += (double)Q[(size_t)k * n + v] + (double)Q[(size_t)v * n + k];
            f[k] = s;
        }
        for (uint64_t i = j->i0;; i++) {
            if (!j->have || E < j->bestEf || (E == j->bestEf && row < j->bestIdx)) {
                j->have = 1;
                j->bestEf = E;
                j->bestIdx = row;
            }
            if (i + 1 >= j->i1) break;
            int t = __builtin_ctzll(i + 1);
            int k = n - 1 - t;
            double d = x[k] ? -1.0 : 1.0;
            E += d * f[k];
            x[k] ^= 1;
            row ^= 1ull << t;
            for (int v = 0; v < n; v++)
                if (v != k) f[v] += d * ((double)Q[(size_t)v * n + k] + (double)Q[(size_t)k * n + v]);
        }
    }
    return NULL;
}

static int o2_solve(int n, const void *Q, int is_int, int threads, int64_t *Ei, double *Ef,
                    uint64_t *idx)
{
    if (n < 1 || n > 62 || !Q || !idx) return -1;
    uint64_t total = 1ull << n;
    int T = resolve_threads(threads, total);
    o2_job_t *jobs = (o2_job_t *)calloc((size_t)T, sizeof(o2_job_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    if (!jobs || !tid) { free(jobs); free(tid); return -2; }
    uint64_t per = total / (uint64_t)T, rem = total % (uint64_t)T, at = 0;
    for (int t = 0; t < T; t++) {
        jobs[t].n = n;
        jobs[t].is_int = is_int;
        jobs[t].Q = Q;
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
    return 0;
}

int oracle_gray_i(int n, const int32_t *Q, int threads, int64_t *E, uint64_t *idx)
{
    if (!E) return -1;
    return o2_solve(n, Q, 1, threads, E, NULL, idx);
}

int oracle_gray_f(int n, const float *Q, int threads, double *E, uint64_t *idx)
{
    if (!E) return -1;
    return o2_solve(n, Q, 0, threads, NULL, E, idx);
}

/* number of worker threads a call with threads <= 0 uses */
int oracle_default_threads(void)
{
    return resolve_threads(0, UINT64_MAX);
}

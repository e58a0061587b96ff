/*
 * qubo.h -- C ABI of the MI355X exhaustive dense-QUBO solver.
 *
 * The solver minimises the QUBO objective E(x) = sum_{i,j} Q_ij x_i x_j over
 * all 2^n binary states x (paper: Introduction; Sec. II-A, Eq. total_energy)
 * by the prefix-suffix decomposition of Sec. II-A/II-C (Eqs.
 * energy_decomposition and chunk_energy_final) and the Gray-code walk of
 * Sec. III-B (Eq. incremental_update, Alg. 2), on int32 vector ALUs of a
 * gfx950 GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Q is a dense row-major n x n matrix, int32 (QUBO_INT32) or float32
 *   (QUBO_FP32).  E sums over ALL i, j, so an upper-triangular Q (the paper's
 *   Sec. II-A form) is the special case with a zero lower triangle; any lower
 *   entries are folded onto the upper triangle.
 * - A state is identified by its "index": its row in the lexicographic state
 *   matrix U_N of Sec. II-B, whose column 0 is the most significant bit:
 *       x_i = (index >> (n - 1 - i)) & 1.
 * - The answer is the lexicographic minimum of (E, index): the minimum energy
 *   and, among the states reaching it, the LOWEST index.  (Alg. 2 keeps the
 *   first state visited in Gray order; this library resolves ties by index.)
 * - 1 <= n <= 60.
 * - int32 input: solved exactly.  The library folds T_ii = Q_ii,
 *   T_ij = Q_ij + Q_ji (i < j) and requires sum_{i<=j} |T_ij| <= 2^30 - 1,
 *   which proves every partial sum the walk forms fits int32 (the paper's
 *   Sec. IV-B.5 overflow pre-check is heuristic; this bound is rigorous).
 *   Larger inputs return QUBO_EOVERFLOW.
 * - float32 input (the paper's Sec. VI-B future work): T is scaled by 2^p and
 *   rounded half-to-even to int32 so that sum |T~| <= 2^29, solved exactly in
 *   int32, and the returned state is rescored in float64 from the caller's Q.
 *   With eps_q = nnz(T) * 2^(-p-1), |E(x) - 2^-p E~(x)| <= eps_q for every x,
 *   so the returned energy is within tol = 2 eps_q of the true minimum.
 *   NaN or Inf entries return QUBO_ENONFINITE.
 * - Inputs are borrowed and read-only; they need to stay valid only for the
 *   duration of the call (qubo_server_submit copies Q before returning).
 * - Outputs are caller-allocated and written only when QUBO_OK is returned.
 * - No C++ exception crosses this ABI.  On error the status is returned and a
 *   thread-local message is available from qubo_last_error().
 * - Every entry point is reentrant; a server handle is internally
 *   synchronised.
 */
#ifndef QUBO_MI355X_H
#define QUBO_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { QUBO_INT32 = 0, QUBO_FP32 = 1 } qubo_dtype_t;

typedef enum {
    QUBO_OK = 0,
    QUBO_EINVAL = -1,      /* bad argument (n out of range, null pointer, bad option) */
    QUBO_EOVERFLOW = -2,   /* int32 input whose |T| sum exceeds 2^30 - 1             */
    QUBO_ENONFINITE = -3,  /* float32 input holding NaN or Inf                        */
    QUBO_ENOMEM = -4,      /* host or device allocation failed                        */
    QUBO_EDEVICE = -5,     /* HIP runtime error (message in qubo_last_error)          */
    QUBO_EAGAIN = -6,      /* server: result not ready yet / admission deferred       */
    QUBO_EINTERNAL = -7    /* a self-check failed (e.g. the argmin rescan)            */
} qubo_status_t;

/* One state with its energy.
 * int32 input : energy_i is the exact energy, energy == (double)energy_i.
 * float32 input: energy is E(x) in float64 from the caller's Q; energy_i is the
 *                scaled integer energy E~(x) = round(2^p T) summed exactly. */
typedef struct {
    int64_t energy_i;
    double energy;
    uint64_t index;
} qubo_state_t;

typedef struct {
    qubo_state_t best;
    double tol;          /* 0 for int32; 2 eps_q for float32 (see above)           */
    int p;               /* fixed-point exponent (0 for int32)                     */
    int A, B;            /* prefix / suffix split used (A + B = n); B = 0: direct  */
    int L;               /* log2 Gray steps per work item                          */
    int tier;            /* 0 direct evaluation (n <= 14); 1 exact lane-min every
                            Gray step; 2 block lower bound, exact min on demand;
                            3 tier 2's test against a top-k threshold (k > 1);
                            4 tier 2 on packed 16-bit chunk energies, two per
                            32-bit word (Sec. IV-B "Data types"); 5 tier 3
                            on the packed layout (k > 1)                   */
    int vgpr_levels;     /* Gray levels with VGPR-resident rows (0 when direct)    */
    uint64_t states;     /* states evaluated = 2^n                                 */
    double kernel_ms;    /* GPU time of the walk kernel (HIP events)               */
    double total_ms;     /* host wall time of the whole call                       */
} qubo_result_t;

/* Plan overrides, mainly for tests and the autotuner.  Zero-initialise for the
 * defaults.  B: suffix bits in [6, 10] (0 = default 10; [9, 11] with tier 4);
 * L: log2 Gray steps per work item in [6, A] (0 = default); tier: 0 = default,
 * 1, 2 or 4 to force that walk tier; waves_per_cu: resident walk waves per
 * compute unit (0 = the occupancy limit); vgpr_levels: see below.
 * Tier 4 (packed) holds two 16-bit chunk energies in each 32-bit word, so one
 * int32 add moves two states.  It is exact whenever the chunk energies
 * E_sd(s, x_p) of the split, over every prefix x_p and suffix column s, span
 * at most 65536 consecutive values (the planner computes their exact
 * extremes and shifts them by a constant c into the signed 16-bit range),
 * and sum |T| + |c| <= 2^30 - 1.  (The int32 walk shifts its chunk energies
 * too, to start at 0: c is reported in qubo_plan_info_t::pack_shift.)  It needs int32 input given in host memory,
 * n - B >= 6 and B - 7 = log2 of a built words-per-lane count (4, 8 or 16);
 * with k > 1 the packed plan runs the top-k walk as tier 5.
 * The default plan (no override) takes it wherever that holds, one suffix
 * bit wider than the int32 plan; forcing it where it does not hold returns
 * QUBO_EINVAL.
 * item_first, item_count: walk only work items [item_first, item_first +
 * item_count) of the plan (item_count 0 = all).  Work item c covers the prefix
 * rows of Gray steps [c 2^L, (c+1) 2^L), which are the aligned block of rows
 * [g(c) 2^L, (g(c)+1) 2^L) with g(c) = c ^ (c >> 1), i.e. the contiguous index
 * range [g(c) 2^(L+B), (g(c)+1) 2^(L+B)); the result is the minimum (and top-k)
 * over the chosen items' states.  For sampled checks at full size; not
 * allowed for direct (n <= 14) plans or in batches. */
typedef struct {
    int B;
    int L;
    int tier;
    int waves_per_cu;
    int vgpr_levels;     /* Gray levels whose M_int rows stay in VGPRs: 0 = default
                            (4 for B = 10, else 12), 12, 8 (B = 9 or 10), 6, 5,
                            4 or 3 (B = 10); fewer levels free VGPRs for a third
                            or fourth wave per SIMD, the higher rows being read
                            from L2 when they flip.  4 keeps levels 0-2 and 5
                            in VGPRs and levels 3-4 in LDS (8 KB per wave); 3
                            keeps levels 0-2 in VGPRs, levels 3-4 in LDS and
                            reads every level from 5 up from L2              */
    int item_first;
    int item_count;
    int reserved;
} qubo_options_t;

/* Solve one instance held in HOST memory.  k = 0 or 1: best state only
 * (topk may be NULL).  k > 1 (the k lowest energies, an extension the paper
 * names in Sec. VI): additionally the k lexicographically smallest
 * (E, index) pairs into topk[0..k-1], ascending (2 <= k <= 1024, k <= 2^n),
 * and out->best = topk[0].  The walk then runs tier 3, or tier 5 on the
 * packed layout (per-wave candidate lists of chunk keys; a selection of the
 * k smallest chunks, their rescan and a selection of the k smallest states
 * finish it).  int32: exact.
 * float32: the k smallest scaled integer energies, reported with their
 * float64 energies and ordered by (energy, index); the i-th reported energy
 * is within out->tol of the exact i-th smallest energy.  Batches and the
 * server return the best state only.  Uses the current HIP device and a
 * stream of the calling thread.  Errors: QUBO_EINVAL for a bad k (checked
 * before any device work). */
qubo_status_t qubo_solve(const void *Q, int n, qubo_dtype_t dtype, int k,
                         qubo_result_t *out, qubo_state_t *topk);

/* As qubo_solve, with plan overrides (opt may be NULL). */
qubo_status_t qubo_solve_ex(const void *Q, int n, qubo_dtype_t dtype, int k,
                            const qubo_options_t *opt, qubo_result_t *out,
                            qubo_state_t *topk);

/* Solve one instance whose Q is already in DEVICE memory of the current HIP
 * device (e.g. a torch tensor's data_ptr), ordering all work on hip_stream
 * (a hipStream_t; NULL = the null stream).  Q is read only on the device:
 * the fold, the int32 exactness proof and the float32 fixed-point scaling run
 * in a kernel ordered after whatever wrote dQ on that stream, with the same
 * arithmetic (and so the same T, p and answer) as qubo_solve on a host copy.
 * The plan is made from n and dtype alone, before any value is read, so it
 * is qubo_solve's except that it never takes the packed tier (4), whose
 * eligibility depends on the values.  Returns after the result has been copied back (the stream is
 * synchronised once, at the end); input errors (QUBO_EOVERFLOW,
 * QUBO_ENONFINITE) are detected on the device and reported then, after a
 * walk that skips every item. */
qubo_status_t qubo_solve_device(const void *dQ, int n, qubo_dtype_t dtype, int k,
                                void *hip_stream, qubo_result_t *out,
                                qubo_state_t *topk);

/* Allocation-free variant of qubo_solve with k = 1, for callers that cannot
 * allocate device memory (code that runs under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same plan, kernels and
 * result as qubo_solve(Q, n, dtype, 1, out, NULL).  Q: host memory as for
 * qubo_solve; work is ordered on hip_stream (a hipStream_t; NULL = the null
 * stream) and the call returns after synchronising it.  The job's device
 * memory is a fixed scratch array of qubo_noalloc_scratch_bytes() bytes
 * (16 MiB) that the library holds on each device it runs on until the
 * process ends; the call makes no device or pinned-host allocation
 * (hipMalloc, hipMallocAsync, hipHostMalloc or a library routine that
 * allocates) and no hipFree.  A plan whose device image exceeds the scratch
 * (large n: the item records grow with the work items) returns QUBO_ENOMEM
 * with the sizes in qubo_last_error().  Every call on one device shares that
 * device's scratch and leaves its contents behind; calls that overlap on one
 * device (another thread, or another stream before this call returns) race
 * and must be serialised by the caller. */
qubo_status_t qubo_solve_noalloc(const void *Q, int n, qubo_dtype_t dtype, void *hip_stream,
                                 qubo_result_t *out);

/* Size in bytes of qubo_solve_noalloc's per-device scratch array. */
size_t qubo_noalloc_scratch_bytes(void);

/* Solve `count` independent instances (host memory) in one persistent walk
 * launch.  Q[i] is n[i] x n[i] of dtype[i].  out[i] receives instance i's
 * result (best state only).  The whole sequence is replayed from a HIP graph. */
qubo_status_t qubo_solve_batch(int count, const void *const *Q, const int *n,
                               const qubo_dtype_t *dtype, qubo_result_t *out);

/* Batch handle: plan, allocate and capture once, replay many times. */
typedef struct qubo_batch qubo_batch_t;
qubo_status_t qubo_batch_create(int count, const void *const *Q, const int *n,
                                const qubo_dtype_t *dtype, const qubo_options_t *opt,
                                qubo_batch_t **batch);
/* Replay the captured graph on hip_stream (NULL = the batch's own stream) and
 * wait for it. */
qubo_status_t qubo_batch_run(qubo_batch_t *batch, void *hip_stream);
qubo_status_t qubo_batch_results(qubo_batch_t *batch, qubo_result_t *out);
/* Total states of the batch and the walk-kernel time of the last replay. */
qubo_status_t qubo_batch_stats(qubo_batch_t *batch, double *states, double *kernel_ms);
void qubo_batch_destroy(qubo_batch_t *batch);

/* Outer-bit reduction (Sec. III-C.1, straightforward parallelisation; used
 * in Sec. IV-C beyond the kernel's size limit).  Fixing the first k variables
 * to xf (variable i < k is bit k-1-i of xf, i.e. xf holds the top k bits of
 * the index) leaves the QUBO of the other m = n - k variables
 *     Qr = T_rr + diag(x_f T_fr),   c = x_f T_ff x_f^T,
 * with T the folded upper-triangular form of Q, so that for every x_r
 * E(x_f, x_r) = c + E_Qr(x_r).  Q: int32 n x n row-major (host); Qr:
 * caller's m x m int32 buffer (upper-triangular on return); c: the constant.
 * 2 <= n <= 64, 1 <= k < n, xf < 2^k (QUBO_EINVAL); QUBO_EOVERFLOW if an
 * entry of Qr leaves int32. */
qubo_status_t qubo_reduce_outer(const int32_t *Q, int n, int k, uint64_t xf,
                                int32_t *Qr, int64_t *c);

/* Solve by outer reduction: the 2^k reduced instances (qubo_reduce_outer)
 * run as one batch, and the answer is the lexicographic minimum of
 * (c(x_f) + E'_min, x_f 2^(n-k) + index'), the same (E, lowest index) as a
 * direct solve.  Extends n to 64 (each reduced instance has n - k <= 60
 * variables).  int32 input only (QUBO_EINVAL otherwise); 2 <= n <= 64,
 * 1 <= k <= 12, 1 <= n - k <= 60.  out: the best state and the first
 * reduced instance's plan fields; states = 2^n (saturated at n = 64);
 * kernel_ms = the batch's walk time. */
qubo_status_t qubo_solve_outer(const void *Q, int n, qubo_dtype_t dtype, int k,
                               qubo_result_t *out);

/* Continuous-batching server (see the serving notes in the docs):
 * requests are admitted into device slots as slots and the device-memory
 * budget allow; each scheduler tick launches one walk over pending work items
 * of every admitted request, so arrivals join work already on the GPU. */
typedef struct qubo_server qubo_server_t;
qubo_status_t qubo_server_create(size_t mem_budget_bytes, int max_slots,
                                 qubo_server_t **srv);
/* Copies Q; returns a ticket.  QUBO_EAGAIN never happens here: admission is
 * deferred inside the server when slots or memory are short. */
qubo_status_t qubo_server_submit(qubo_server_t *srv, const void *Q, int n,
                                 qubo_dtype_t dtype, uint64_t *ticket);
/* QUBO_OK with the result once finished, QUBO_EAGAIN while pending. */
qubo_status_t qubo_server_poll(qubo_server_t *srv, uint64_t ticket, qubo_result_t *out);
/* Blocks until the ticket finishes or timeout_ms passes (QUBO_EAGAIN). */
qubo_status_t qubo_server_wait(qubo_server_t *srv, uint64_t ticket, double timeout_ms,
                               qubo_result_t *out);
/* Latency percentiles over finished requests (arrival -> result ready) and
 * aggregate states/s since creation. */
qubo_status_t qubo_server_stats(qubo_server_t *srv, double *p50_ms, double *p99_ms,
                                double *states_per_s);
/* Scheduler counters: device memory held by admitted requests now and at
 * its peak, the peak number of admitted requests, and walk ticks launched. */
qubo_status_t qubo_server_info(qubo_server_t *srv, size_t *mem_in_use, size_t *mem_peak,
                               int *active_peak, uint64_t *ticks);
/* Stops accepting work, finishes every submitted request, frees the server. */
void qubo_server_destroy(qubo_server_t *srv);

/* ------------------------------------------------------- long solves
 * Very large n (a walk of minutes to hours) in bounded slices with a
 * resumable checkpoint.  The search space splits into independent segments
 * whose minima reduce to the global one (the map-reduce scheme of Sec.
 * III-C, which Sec. IV-C applies beyond the kernel's size limit).  Here a
 * segment is a run of the plan's work items (see qubo_options_t): the solve
 * walks items [next_item, next_item + items_per_slice) per slice, folds each
 * slice's (E, index) into the running lexicographic minimum and then
 * rewrites the checkpoint file at `path` (a sibling "<path>.tmp" is written
 * and renamed over it, so the file is always whole).  If `path` already
 * holds a checkpoint, the solve resumes after its last finished slice.
 *
 * Q, n, dtype: as qubo_solve.  opt (may be NULL): plan overrides as for
 * qubo_solve_ex; item_first / item_count must be 0.  A resumed solve keeps
 * the plan recorded in the checkpoint; an override that contradicts it is
 * QUBO_EINVAL.  items_per_slice: work items per slice (0 = all remaining
 * items in one slice; n <= 14 plans are always one slice).  max_slices: stop
 * after this many slices in this call (0 = run to the end).
 * Returns QUBO_OK with *out = the final result once every item is done
 * (states = 2^n; kernel_ms = walk time summed over all slices of all calls;
 * total_ms = this call), QUBO_EAGAIN when max_slices slices ran and items
 * remain (*out untouched: read progress with qubo_checkpoint_info), and
 * QUBO_EINVAL for a checkpoint that is malformed, belongs to another input
 * (n, dtype or the FNV-1a hash of Q differ) or cannot be written.  The
 * result equals qubo_solve's for the same input and plan.  Calls that share
 * one path at the same time race. */
typedef struct {
    int n;
    qubo_dtype_t dtype;
    int A, B, L, tier, vgpr_levels;   /* plan of every slice (B = 0: direct)   */
    uint64_t q_hash;      /* FNV-1a 64 of n, dtype and the n*n input words     */
    uint64_t items;       /* work items of the plan (1 for a direct plan)      */
    uint64_t next_item;   /* items [0, next_item) are finished                 */
    int found;            /* 1 once best holds a state (next_item > 0)         */
    qubo_state_t best;    /* lexicographic minimum over the finished items     */
    int p;                /* fixed-point exponent (float32 input)              */
    double tol;           /* as qubo_result_t.tol                              */
    double walk_ms;       /* walk-kernel time summed over finished slices      */
} qubo_checkpoint_t;

qubo_status_t qubo_solve_checkpointed(const void *Q, int n, qubo_dtype_t dtype,
                                      const qubo_options_t *opt, uint64_t items_per_slice,
                                      int max_slices, const char *path, qubo_result_t *out);

/* Read a checkpoint written by qubo_solve_checkpointed (host only, never
 * touches the GPU).  QUBO_EINVAL if the file is missing or malformed. */
qubo_status_t qubo_checkpoint_info(const char *path, qubo_checkpoint_t *info);

/* Measurement: int32 VALU throughput of this device.  Runs wave64 streams of
 * independent `op` instructions (0: v_add_u32, 1: v_min3_i32, 2: v_add_u32
 * with one scalar add per two vector adds, 3: v_add_u32 with one never-taken
 * scalar compare-and-branch per 16 vector adds, 4: v_pk_add_u16, 5:
 * v_pk_min_i16, 6: v_add_u32 with a register footprint that admits at most 3
 * waves per SIMD, 7: v_add_f32) with waves_per_simd resident waves on every
 * SIMD and reports
 * vector lane-operations per second (a packed instruction counts once per
 * lane) and the kernel time. */
qubo_status_t qubo_probe_valu(int op, int waves_per_simd, int iters, double *lane_ops_per_s,
                              double *ms);

/* Host-only planning, for tests: fold, overflow proof / fp32 scale, split.
 * Never touches the GPU.  T_out (n*n int32, may be NULL) receives the folded
 * (and for float32 scaled) upper-triangular matrix the kernels consume. */
typedef struct {
    int n, A, B, L, tier, direct, vgpr_levels;
    int p;
    double eps_q;
    int64_t sum_abs_t;   /* sum |T~_ij| over i <= j */
    uint64_t items;      /* walk work items */
    int pack_shift;      /* tier 4: the constant c added to every chunk energy
                            (taken off every prefix energy) so that each fits
                            a signed 16-bit value; 0 otherwise */
    int reserved;
} qubo_plan_info_t;
qubo_status_t qubo_plan_info(const void *Q, int n, qubo_dtype_t dtype,
                             const qubo_options_t *opt, qubo_plan_info_t *info,
                             int32_t *T_out);

/* ---------------------------------------------------------------- tuning
 * The walk has knobs whose best setting depends on n and on the device: the
 * suffix width B (columns per lane), the row-cache depth vgpr_levels, the
 * bound tier and the work-item size L.  The paper tuned its kernel by hand
 * on its GPU (Sec. IV); here the library times every plan it can run and
 * keeps the fastest per (scope, n, dtype) in a process-wide table that the
 * planner consults whenever the caller's options override none of B, L, tier
 * and vgpr_levels (all zero or opt == NULL).  Two scopes: QUBO_TUNE_SINGLE
 * entries (qubo_autotune) serve lone solves, whose speed depends on spreading
 * one instance over the GPU; QUBO_TUNE_BATCH entries (qubo_autotune_batch)
 * serve instances of batches and the server, where many instances fill the
 * GPU (their L is always the batch item size).  The table starts empty
 * (built-in defaults) unless QUBO_TUNE_CACHE names a cache file, which is
 * then loaded at the first solve, batch or server submission. */
#define QUBO_TUNE_SINGLE 0
#define QUBO_TUNE_BATCH 1
typedef struct {
    int n;                 /* variables, 15..60                                  */
    qubo_dtype_t dtype;
    int B, L, tier, vgpr_levels;   /* L = 0: the planner's default item size
                                      (always 0 for QUBO_TUNE_BATCH)          */
    double walk_ms;        /* measured time of this plan (informational): the
                              walk kernel for single entries, one batch replay
                              for batch entries                              */
    int scope;             /* QUBO_TUNE_SINGLE or QUBO_TUNE_BATCH               */
} qubo_tune_entry_t;

/* Time every runnable plan for each n in [n_min, n_max] (15 <= n_min <= n_max
 * <= 48) on a synthetic instance of `dtype` on the current device: each
 * candidate once, then the four fastest `reps` more times (minimum kept).
 * Fails with QUBO_EINTERNAL if two plans disagree on (E*, index*).  The
 * winners go into the process table; with cache_path they are also merged
 * into that JSON file (created if absent; entries made for this device that it
 * already holds are kept unless re-tuned).  out[0..min(out_cap, count)-1]
 * receive the winners in n order and *out_count their number (both may be
 * NULL / 0).  Cost: about 60 solves per n, dominated by the largest n. */
qubo_status_t qubo_autotune(int n_min, int n_max, qubo_dtype_t dtype, int reps,
                            const char *cache_path, qubo_tune_entry_t *out,
                            int out_cap, int *out_count);

/* The batch-scope counterpart of qubo_autotune: for each n in [n_min, n_max]
 * (15 <= n_min <= n_max <= 44) it times every runnable (B, vgpr_levels, tier)
 * on a batch of m = min(4096, max(1, 2^(39-n))) copies of the synthetic
 * instance -- enough work to fill the GPU, as in the batch and server
 * workloads -- by the event time of one graph replay, each candidate once and
 * the four fastest `reps` more times.  The built-in plan is kept unless a
 * candidate is at least 5% faster (each extra kernel variant in a batch adds
 * a persistent launch and its tail, which a per-n timing does not see).
 * Every instance of every candidate must return the same (E*, index*)
 * (QUBO_EINTERNAL otherwise).  Winners go into the table with scope
 * QUBO_TUNE_BATCH and, with cache_path, into that file, as for
 * qubo_autotune. */
qubo_status_t qubo_autotune_batch(int n_min, int n_max, qubo_dtype_t dtype, int reps,
                                  const char *cache_path, qubo_tune_entry_t *out,
                                  int out_cap, int *out_count);

/* Load a cache file into the process table.  device_key: the key the file
 * must carry; NULL = this device's key (qubo_device_key).  A file made on
 * another device, malformed JSON or an entry naming a plan the library's kernels cannot
 * run is rejected as a whole with QUBO_EINVAL.  *loaded = entries read. */
qubo_status_t qubo_tune_load(const char *path, const char *device_key, int *loaded);

/* Write the whole process table to path under device_key (NULL = this
 * device's key), replacing the file. */
qubo_status_t qubo_tune_save(const char *path, const char *device_key);

/* Put entries into the process table directly (validated as by
 * qubo_tune_load; nothing is stored if any entry is invalid). */
qubo_status_t qubo_tune_set(const qubo_tune_entry_t *entries, int count);

/* 1 and *out filled (out may be NULL) if the table holds (scope, n, dtype),
 * else 0. */
int qubo_tune_lookup(int n, qubo_dtype_t dtype, int scope, qubo_tune_entry_t *out);

/* Empty the process table (built-in defaults again). */
void qubo_tune_clear(void);

/* This device's cache key, "<gfx arch>/<compute units>cu", e.g. "gfx950/256cu". */
qubo_status_t qubo_device_key(char *buf, int cap);

/* Thread-local description of the last error on this thread ("" if none). */
const char *qubo_last_error(void);

/* Library version string. */
const char *qubo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QUBO_MI355X_H */

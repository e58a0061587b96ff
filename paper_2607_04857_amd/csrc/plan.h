// plan.h -- host-side planning of one QUBO solve (no HIP dependency).
//
// Step "canonicalise and plan": fold Q into the upper-triangular T the
// paper's decomposition assumes (Sec. II-A), prove int32 is exact or scale a
// float32 Q to fixed point, and choose the prefix/suffix split
// (A + B = N, Sec. II-A) and the work-item size of the Gray walk.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qubo.h"

namespace qplan {

// Kernel geometry shared by planner and kernels.
constexpr int kWave = 64;          // lanes per wavefront
constexpr int kSuper = 6;          // log2 of the unrolled Gray super-block (64 steps)
constexpr int kManyMinL = 10;      // log2 of the shortest item of an instance in a batch or
                                   // the server (4096 copies of n = 22: 4.0 ms per replay
                                   // with 2^6-step items, 1.3 ms with 2^10-step ones)
constexpr int kMaxN = 60;
constexpr int kDirectMaxN = 14;    // n at or below this: direct evaluation, no walk
constexpr int64_t kIntSumLimit = (int64_t(1) << 30) - 1;   // sum |T| bound, int32 input
constexpr double kFpScaleTarget = double(int64_t(1) << 29); // sum |T~| target, fp32 input
constexpr int64_t kPackSumLimit = (int64_t(1) << 15) - 1;    // suffix-column sum |T|, tier 4

struct Plan {
    int n = 0;
    qubo_dtype_t dtype = QUBO_INT32;
    bool direct = false;   // evaluate all 2^n states directly (tiny n)
    int A = 0, B = 0;      // prefix / suffix bits
    int mcols = 0;         // suffix columns per lane = 2^B / 64
    int L = 0;             // log2 Gray steps per work item
    int tier = 0;          // 0 direct; 1: exact lane-min each step; 2: block lower bound;
                           // 4: tier 2 on packed 16-bit chunk energies;
                           // 3 / 5: top-k lists on the int32 / packed walk
                           // (set by the top-k planning)
    int vgpr_levels = 0;   // Gray levels whose M_int rows are VGPR-resident
    int32_t pack_shift = 0;   // c added to every chunk energy (and subtracted
                              // from every prefix energy): tiers 4, 5 centre
                              // them in 16 bits, the int32 walk starts them
                              // at 0 (fewer result bits toggle per add)
    int p = 0;             // fixed-point exponent (fp32)
    double eps_q = 0.0;    // per-state quantisation bound (fp32)
    int64_t sum_abs = 0;   // sum |T| over i <= j (of the int32 matrix solved)
    uint64_t items = 0;    // 2^(A - L) walk items (0 when direct)
    uint64_t item_first = 0, item_count = 0;   // walk only these items (count 0: all)
    uint64_t walk_items() const { return item_count ? item_count : items; }
    std::vector<int32_t> T;    // folded (and scaled) upper-triangular n x n
};

// One tuned walk choice for instances of n variables and a dtype.
// Scope of an entry: the plan of a lone solve (its latency: every item of
// one instance spread over the GPU), or the plan of an instance inside a
// batch or the server (throughput: the GPU filled by many instances).
constexpr int kScopeSingle = 0;
constexpr int kScopeBatch = 1;

struct TuneEntry {
    int n = 0;
    qubo_dtype_t dtype = QUBO_INT32;
    int B = 0, L = 0, tier = 0, vgpr_levels = 0;
    double walk_ms = 0.0;      // measured walk time of the chosen plan
    int scope = kScopeSingle;
};

// Process-wide tuning table (thread-safe), keyed by (scope, n, dtype).
// make_plan consults it when the caller overrides none of B, L, tier and
// vgpr_levels: the single scope for lone solves, the batch scope for
// instances of batches and the server.
void tune_put(const TuneEntry &e);
bool tune_get(int n, qubo_dtype_t dtype, int scope, TuneEntry *out);
void tune_clear();
std::vector<TuneEntry> tune_all();

// Check that a tuning entry describes a plan whose kernel variant the library compiles.
bool tune_valid(const TuneEntry &e, std::string *msg);

// Build a plan from a host Q.  Returns QUBO_OK or an error with msg set.
// `many`: the instance shares its walk launch with others (batch, server),
// so it needs no item-level parallelism of its own (a tuned L is then
// ignored: it was measured for a lone instance).  `packed_ok`: the plan may
// take the packed tier (4) where the input allows it.
qubo_status_t make_plan(const void *Q, int n, qubo_dtype_t dtype, const qubo_options_t *opt,
                        Plan *out, std::string *msg, bool many = false, bool packed_ok = true);

// Sum of |T_ij| over the columns j >= A (i <= j): a bound on |E_sd| of every
// chunk of the split at A.
int64_t suffix_sum_abs(const Plan &P, int A);

// Exact extremes, over every prefix and suffix column, of the chunk energies
// E_sd of the split at A (P.T set).
void chunk_energy_range(const Plan &P, int A, int64_t *lo, int64_t *hi);

// Whether the split at A can run the packed tier, and its shift c: every
// E_sd + c must be a signed 16-bit value, the least one -2^15 (from the
// exact range), and P.sum_abs + |c| must stay within kIntSumLimit (the
// prefix energies move by -c).
bool packed_shift(const Plan &P, int A, int32_t *shift);

// Shift of the int32 walk at the split A: c = -(least chunk energy), so every
// E_sd + c is non-negative (the sum's upper bits then stay 0 instead of
// flipping with the sign, which draws less power per add and lets the chip
// hold a higher clock; measured 5% on the n = 44 walk), or 0 where P.sum_abs
// + |c| would leave the int32 bound.
int32_t nonneg_shift(const Plan &P, int A);

// The walk plan of an instance whose values are not on the host (a lone
// solve of a device-resident Q): as make_plan, except that T, p, eps_q and
// sum_abs are left for the device to fill (the plan does not depend on them).
qubo_status_t make_plan_shape(int n, qubo_dtype_t dtype, const qubo_options_t *opt, Plan *out,
                              std::string *msg);

// Fixed-point exponent of a float32 input: the largest p with S 2^p <= 2^29
// for S = sum |T_ij| > 0 (0 for S = 0), exactly (from S's binary exponent).
int fp_scale_exponent(double S);

}  // namespace qplan

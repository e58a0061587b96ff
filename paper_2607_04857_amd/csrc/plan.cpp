// plan.cpp -- fold, exactness proof / fixed-point scale, split and work items.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

namespace qplan {

namespace {

// Default suffix width: 64 lanes x 16 columns (B = 10) keeps the lane's
// columns and the twelve most frequently flipped M_int rows in VGPRs.
constexpr int kDefaultB = 10;
constexpr int kMinB = 6;           // one column per lane
constexpr int kMaxB = 10;          // 16 columns per lane (VGPR budget)
constexpr int kDefaultTier = 2;

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, TuneEntry> g_tune;   // (scope, n, dtype) -> entry

bool variant_built(int mcols, int G)
{
    if (G == 12) return mcols == 1 || mcols == 2 || mcols == 4 || mcols == 8 || mcols == 16;
    if (G == 8) return mcols == 8 || mcols == 16;
    if (G == 6 || G == 5 || G == 4 || G == 3) return mcols == 16;
    return false;
}

}  // namespace

void tune_put(const TuneEntry &e)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(e.scope, e.n, int(e.dtype))] = e;
}

bool tune_get(int n, qubo_dtype_t dtype, int scope, TuneEntry *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(scope, n, int(dtype)));
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

void tune_clear()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

std::vector<TuneEntry> tune_all()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::vector<TuneEntry> v;
    for (const auto &kv : g_tune) v.push_back(kv.second);
    return v;
}

bool tune_valid(const TuneEntry &e, std::string *msg)
{
    if (e.n <= kDirectMaxN || e.n > kMaxN) {
        *msg = "tuning entry n must be in [15, 60]";
        return false;
    }
    if (e.dtype != QUBO_INT32 && e.dtype != QUBO_FP32) {
        *msg = "tuning entry has an unknown dtype";
        return false;
    }
    if (e.B < kMinB || e.B > kMaxB || e.n - e.B < kSuper) {
        *msg = "tuning entry B must be in [6, 10] with n - B >= 5";
        return false;
    }
    if (e.tier != 1 && e.tier != 2) {
        *msg = "tuning entry tier must be 1 or 2";
        return false;
    }
    if (e.scope != kScopeSingle && e.scope != kScopeBatch) {
        *msg = "tuning entry scope must be single (0) or batch (1)";
        return false;
    }
    if (e.scope == kScopeBatch && e.L != 0) {
        *msg = "batch tuning entries keep the batch item size (L = 0)";
        return false;
    }
    if (!variant_built((1 << e.B) / kWave, e.vgpr_levels)) {
        *msg = "tuning entry names a (B, vgpr_levels) walk variant that is not built";
        return false;
    }
    const int A = e.n - e.B;
    if (e.L != 0 && (e.L < kSuper || e.L > A || A - e.L > 20)) {
        *msg = "tuning entry L must be 0 or in [max(6, A - 20), A]";
        return false;
    }
    return true;
}

static_assert(kFpScaleTarget == 536870912.0, "fp_scale_exponent assumes the 2^29 target");

int fp_scale_exponent(double S)
{
    // S = m 2^e with m in [0.5, 1): m 2^(e+p) <= 2^29 holds for e + p <= 29,
    // and for e + p = 30 exactly when m = 0.5
    if (!(S > 0.0)) return 0;
    int e = 0;
    const double m = std::frexp(S, &e);
    return (m == 0.5 ? 30 : 29) - e;
}

static qubo_status_t check_args(int n, qubo_dtype_t dtype, std::string *msg)
{
    if (n < 1 || n > kMaxN) {
        *msg = "n must be in [1, 60]";
        return QUBO_EINVAL;
    }
    if (dtype != QUBO_INT32 && dtype != QUBO_FP32) {
        *msg = "unknown dtype";
        return QUBO_EINVAL;
    }
    return QUBO_OK;
}

static qubo_status_t plan_walk(const qubo_options_t *opt, Plan &P, std::string *msg, bool many,
                               bool packed_ok);

int64_t suffix_sum_abs(const Plan &P, int A)
{
    const size_t nn = size_t(P.n);
    int64_t s = 0;
    for (size_t j = size_t(A); j < nn; j++)
        for (size_t i = 0; i <= j; i++) {
            const int64_t t = P.T[i * nn + j];
            s += t < 0 ? -t : t;
        }
    return s;
}

void chunk_energy_range(const Plan &P, int A, int64_t *lo, int64_t *hi)
{
    const size_t nn = size_t(P.n);
    const int B = P.n - A;
    const size_t NS = size_t(1) << B;
    // E_sd(s, x_p) = E_s(s) + sum_v x_v M[v][s]; over all prefixes x_p its
    // extremes are E_s(s) + the sums of the negative / positive M[v][s].
    // Column s is a subset of the suffix variables (bit b <-> variable
    // A + B-1-b); each array is filled from s with its lowest bit cleared.
    std::vector<int64_t> es(NS, 0), neg(NS, 0), pos(NS, 0), m(NS, 0);
    auto var = [&](size_t s) { return A + B - 1 - __builtin_ctzll(uint64_t(s)); };
    for (size_t s = 1; s < NS; s++) {
        const size_t r = s & (s - 1);
        const size_t w = size_t(var(s));
        int64_t e = es[r] + P.T[w * nn + w];
        for (size_t q = r; q; q &= q - 1) {
            const size_t u = size_t(var(q));
            e += u < w ? P.T[u * nn + w] : P.T[w * nn + u];
        }
        es[s] = e;
    }
    for (int v = 0; v < A; v++) {
        m[0] = 0;
        for (size_t s = 1; s < NS; s++) {
            m[s] = m[s & (s - 1)] + P.T[size_t(v) * nn + size_t(var(s))];
            (m[s] < 0 ? neg[s] : pos[s]) += m[s];
        }
    }
    int64_t l = INT64_MAX, h = INT64_MIN;
    for (size_t s = 0; s < NS; s++) {
        l = std::min(l, es[s] + neg[s]);
        h = std::max(h, es[s] + pos[s]);
    }
    *lo = l;
    *hi = h;
}

int32_t nonneg_shift(const Plan &P, int A)
{
    int64_t lo = 0, hi = 0;
    chunk_energy_range(P, A, &lo, &hi);
    return P.sum_abs + (lo < 0 ? -lo : lo) <= kIntSumLimit ? int32_t(-lo) : 0;
}

bool packed_shift(const Plan &P, int A, int32_t *shift)
{
    // the exact extremes decide (the suffix-column sum, a cheaper bound of
    // them, is not used: the shift below also wants the least value)
    int64_t lo = 0, hi = 0;
    chunk_energy_range(P, A, &lo, &hi);
    if (hi - lo > 2 * kPackSumLimit + 1) return false;
    // shifted chunk energies E_sd + c span [-2^15, hi - lo - 2^15], so the
    // biased halves start at 0 and their upper bits flip as little as the
    // range allows (measured 5% on the packed n = 44 walk against c = 0)
    const int64_t c = -(kPackSumLimit + 1) - lo;
    // the prefix energies (and the thresholds formed from them) move by -c:
    // they stay within the int32 bound's reach
    if (P.sum_abs + (c < 0 ? -c : c) > kIntSumLimit) return false;
    *shift = int32_t(c);
    return true;
}

qubo_status_t make_plan(const void *Q, int n, qubo_dtype_t dtype, const qubo_options_t *opt,
                        Plan *out, std::string *msg, bool many, bool packed_ok)
{
    if (!Q || !out) {
        *msg = "null argument";
        return QUBO_EINVAL;
    }
    qubo_status_t st = check_args(n, dtype, msg);
    if (st != QUBO_OK) return st;
    Plan P;
    P.n = n;
    P.dtype = dtype;
    P.T.assign(size_t(n) * n, 0);
    const size_t nn = size_t(n);

    // Fold: E sums over all (i, j), so T_ii = Q_ii and T_ij = Q_ij + Q_ji for
    // i < j describe the same objective with a zero lower triangle.
    if (dtype == QUBO_INT32) {
        const int32_t *q = static_cast<const int32_t *>(Q);
        int64_t sum = 0;
        for (size_t i = 0; i < nn; i++) {
            for (size_t j = i; j < nn; j++) {
                int64_t t = (i == j) ? int64_t(q[i * nn + i])
                                     : int64_t(q[i * nn + j]) + int64_t(q[j * nn + i]);
                sum += t < 0 ? -t : t;
                if (sum > kIntSumLimit) {
                    *msg = "sum of |T_ij| exceeds 2^30 - 1: int32 walk not provably exact";
                    return QUBO_EOVERFLOW;
                }
                P.T[i * nn + j] = int32_t(t);
            }
        }
        P.sum_abs = sum;
    } else {
        const float *q = static_cast<const float *>(Q);
        std::vector<double> Td(nn * nn, 0.0);
        double S = 0.0;
        int nnz = 0;
        for (size_t i = 0; i < nn; i++) {
            for (size_t j = i; j < nn; j++) {
                double a = q[i * nn + j], b = (i == j) ? 0.0 : double(q[j * nn + i]);
                if (!std::isfinite(a) || !std::isfinite(b)) {
                    *msg = "non-finite entry in Q";
                    return QUBO_ENONFINITE;
                }
                double t = a + b;
                Td[i * nn + j] = t;
                S += std::fabs(t);
                if (t != 0.0) nnz++;
            }
        }
        // Largest p with S * 2^p <= 2^29; every partial sum of T~ then stays
        // within 2^29 + nnz / 2 < 2^30 - 1.
        const int p = fp_scale_exponent(S);
        int64_t sum = 0;
        for (size_t i = 0; i < nn; i++)
            for (size_t j = i; j < nn; j++) {
                double v = std::nearbyint(std::ldexp(Td[i * nn + j], p));  // ties to even
                int64_t t = int64_t(v);
                P.T[i * nn + j] = int32_t(t);
                sum += t < 0 ? -t : t;
            }
        if (sum > kIntSumLimit) {
            *msg = "internal: scaled matrix exceeds the int32 bound";
            return QUBO_EINTERNAL;
        }
        P.p = p;
        P.sum_abs = sum;
        // Each rounded entry is within 2^(-p-1) of T_ij * 2^p / 2^p, and a
        // state's energy sums at most nnz entries.
        P.eps_q = double(nnz) * std::ldexp(1.0, -p - 1);
    }
    st = plan_walk(opt, P, msg, many, packed_ok && dtype == QUBO_INT32);
    if (st != QUBO_OK) return st;
    *out = std::move(P);
    return QUBO_OK;
}

qubo_status_t make_plan_shape(int n, qubo_dtype_t dtype, const qubo_options_t *opt, Plan *out,
                              std::string *msg)
{
    if (!out) {
        *msg = "null argument";
        return QUBO_EINVAL;
    }
    qubo_status_t st = check_args(n, dtype, msg);
    if (st != QUBO_OK) return st;
    Plan P;
    P.n = n;
    P.dtype = dtype;
    st = plan_walk(opt, P, msg, false, false);
    if (st != QUBO_OK) return st;
    *out = std::move(P);
    return QUBO_OK;
}

// The walk plan of P (n and dtype set; T too when packed_ok): split, tier,
// row cache, items.  packed_ok: the packed tier may be chosen (int32 input
// whose values are on the host).
static qubo_status_t plan_walk(const qubo_options_t *opt, Plan &P, std::string *msg, bool many,
                               bool packed_ok)
{
    const int n = P.n;
    const qubo_dtype_t dtype = P.dtype;
    // A tuned choice applies when the caller overrides none of the walk knobs.
    TuneEntry tuned;
    const bool overridden = opt && (opt->B || opt->L || opt->tier || opt->vgpr_levels);
    const bool use_tune = !overridden && n > kDirectMaxN &&
                          tune_get(n, dtype, many ? kScopeBatch : kScopeSingle, &tuned);

    if (opt && (opt->tier < 0 || opt->tier > 4 || opt->tier == 3)) {
        *msg = "option tier must be 0 (default), 1, 2 or 4";
        return QUBO_EINVAL;
    }
    const bool force_pk = opt && opt->tier == 4;
    if (opt && opt->B && !force_pk && (opt->B < kMinB || opt->B > kMaxB)) {
        *msg = "option B must be in [6, 10]";
        return QUBO_EINVAL;
    }
    if (opt && opt->B && force_pk && (opt->B < kMinB + 3 || opt->B > kMaxB + 1)) {
        *msg = "option B must be in [9, 11] for tier 4";
        return QUBO_EINVAL;
    }
    // B of the int32 walk (tier 4 is then planned one suffix bit wider, the
    // same words per lane holding two columns each)
    int B = (opt && opt->B) ? (force_pk ? opt->B - 1 : opt->B) : (use_tune ? tuned.B : kDefaultB);
    int tier = (opt && opt->tier && !force_pk) ? opt->tier : (use_tune ? tuned.tier : kDefaultTier);
    int vgpr_levels = (opt && opt->vgpr_levels) ? opt->vgpr_levels : (use_tune ? tuned.vgpr_levels : 0);
    if (vgpr_levels != 0 && vgpr_levels != 12 && vgpr_levels != 8 && vgpr_levels != 6 &&
        vgpr_levels != 5 && vgpr_levels != 4 && vgpr_levels != 3) {
        *msg = "option vgpr_levels must be 0, 3, 4, 5, 6, 8 or 12";
        return QUBO_EINVAL;
    }
    P.direct = n <= kDirectMaxN;
    if (!P.direct && n - B < kSuper) B = n - kSuper;  // the prefix must hold one super-block
    if (P.direct) {
        if (opt && (opt->item_first || opt->item_count)) {
            *msg = "item ranges need a walked plan (n > 14)";
            return QUBO_EINVAL;
        }
        P.A = 0;
        P.B = 0;
        P.mcols = 0;
        P.L = 0;
        P.items = 0;
        P.tier = 0;
        return QUBO_OK;
    }
    if (B > kMaxB) B = kMaxB;
    P.B = B;
    P.A = n - B;
    P.mcols = (1 << B) / kWave;
    P.tier = tier;
    // Default row cache for B = 10: levels 0-2 and 5 in VGPRs, 3 and 4 in LDS
    // (four waves per SIMD without spills); all 12 in VGPRs for narrower
    // suffixes.
    if (vgpr_levels == 0) vgpr_levels = P.mcols == 16 ? 4 : 12;
    if ((vgpr_levels == 8 && P.mcols < 8) || (vgpr_levels <= 6 && vgpr_levels && P.mcols != 16)) {
        *msg = force_pk ? "tier 4: vgpr_levels 8 needs B = 10 or 11, vgpr_levels 3, 4, 5 and 6 need B = 11"
                        : "vgpr_levels 8 needs B = 9 or 10, vgpr_levels 3, 4, 5 and 6 need B = 10";
        return QUBO_EINVAL;
    }
    P.vgpr_levels = vgpr_levels;

    // Packed tier (two 16-bit chunk energies per word, one add per two
    // states): for int32 input whose chunk energies provably fit 16 bits at
    // the wider split, chosen by default where it applies, or forced.
    {
        const int Bp = B + 1, Ap = n - Bp;
        const char *why = nullptr;
        int32_t shift = 0;
        if (force_pk && !packed_ok)
            why = "tier 4 needs an int32 matrix given in host memory";
        else if (P.mcols < 4 || !variant_built(P.mcols, vgpr_levels))
            why = "tier 4 needs B = 9, 10 or 11 with a built row cache";
        else if (Ap < kSuper)
            why = "tier 4 needs n - B >= 6";
        else if (packed_ok && !packed_shift(P, Ap, &shift))
            why = "tier 4 needs every chunk energy of the split within a 16-bit range (max - min <= 65535)";
        if (force_pk && why) {
            *msg = why;
            return QUBO_EINVAL;
        }
        const bool auto_pk = !overridden && packed_ok;
        if (!why && (force_pk || auto_pk)) {
            P.B = Bp;
            P.A = Ap;
            P.tier = 4;
            P.pack_shift = shift;
        } else if (!P.T.empty()) {
            P.pack_shift = nonneg_shift(P, P.A);
        }
    }

    // Work items: 2^L consecutive Gray steps each.  Default 2^14 steps (the
    // per-item set-up, about A*MC adds plus the prefix fields, stays below
    // 0.3% of the item), the whole prefix range when it is smaller, and never
    // more than 2^20 items per instance.  A lone instance instead keeps at
    // least 2^13 items (two per resident wavefront) down to 2^9-step items,
    // and at most 2^18 (longer items where there are plenty: fewer item
    // records and set-ups; the autotuner measured this at n = 43 and 44).
    int L;
    if (opt && opt->L) {
        L = opt->L;
        if (L < kSuper || L > P.A) {
            *msg = "option L must be in [6, A]";
            return QUBO_EINVAL;
        }
    } else if (use_tune && tuned.L && !many && tuned.B == P.B) {
        L = tuned.L;
    } else if (use_tune && tuned.L && !many && P.tier == 4 && tuned.B + 1 == P.B) {
        L = std::min(std::max(tuned.L - 1, kSuper), P.A);   // the tuned number of items
    } else {
        L = P.A < 14 ? P.A : 14;
        // An instance sharing the GPU (batch, server) gets up to 64 items
        // where its prefix allows, of at least 2^kManyMinL steps: a small one
        // then finishes on several waves instead of one (server latency), a
        // large one keeps 2^14-step items, and no item is so short that its
        // set-up (finding its instance among thousands, loading that
        // instance's rows, the state from scratch) outweighs its walk.
        if (many && P.A - L < 6) L = std::max(std::min(P.A, kManyMinL), P.A - 6);
        if (!many && P.A - L < 13) L = P.A - 13 < 9 ? 9 : P.A - 13;
        if (!many && P.A - L > 18) L = P.A - 18;
        if (L > P.A) L = P.A;
        if (P.A - L > 20) L = P.A - 20;
    }
    P.L = L;
    P.items = uint64_t(1) << (P.A - L);
    if (opt && (opt->item_first || opt->item_count)) {
        if (opt->item_first < 0 || opt->item_count < 1 ||
            uint64_t(opt->item_first) + uint64_t(opt->item_count) > P.items) {
            *msg = "item range must satisfy 0 <= item_first, 1 <= item_count, first + count <= items";
            return QUBO_EINVAL;
        }
        P.item_first = uint64_t(opt->item_first);
        P.item_count = uint64_t(opt->item_count);
    }
    return QUBO_OK;
}

}  // namespace qplan

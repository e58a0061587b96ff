// tune.cpp -- empirical choice of the walk plan per (n, dtype) and its cache.
//
// The walk has several knobs whose best setting depends on n and on the
// device: the suffix width B (columns per lane, i.e. the wave's block shape),
// the row-cache depth (Gray levels whose M_int rows stay in VGPRs, which
// trades VGPRs for resident waves), the bound tier and the work-item size L.
// The paper reports reaching its kernel's speed by extensive experimentation
// on its GPU (Sec. IV); here that experimentation is a function: time every
// plan the library's kernels can run on a synthetic instance of each n, keep the
// fastest, and let the planner use it.  Every candidate must return the same
// (E*, index*) -- plan invariance is checked on every tuning run.
//
// Two scopes: lone solves are timed by their walk kernel; instances of
// batches and the server by the replay of a batch that fills the GPU, since
// the best plan for one instance spread over the whole GPU (more, smaller
// items: narrower suffixes at small n) is not the best one for many
// instances sharing it.
//
// Cache file: a JSON object
//   {"format": "qubo-tune-1", "device": "<arch>/<CUs>cu",
//    "entries": [{"n": .., "dtype": "int32"|"fp32", "B": .., "L": ..,
//                 "tier": .., "vgpr_levels": .., "walk_ms": ..,
//                 "scope": "single"|"batch"}, ...]}
// (an entry without "scope" is a single-solve entry).
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "hostio.h"
#include "runtime.h"

namespace {

using qhost::format_cache;
using qhost::parse_cache;
using qhost::read_file;
using qhost::write_file;

qubo_status_t current_device_key(std::string *key)
{
    int dev = 0;
    QRT_HIP(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t prop;
    QRT_HIP(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    std::string arch(prop.gcnArchName);
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    *key = arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
    return QUBO_OK;
}

qubo_status_t load_into_table(const char *path, const std::string &key, int *loaded)
{
    std::string text, msg;
    if (!read_file(path, &text, &msg)) {
        qrt::set_error(msg);
        return QUBO_EINVAL;
    }
    std::vector<qplan::TuneEntry> entries;
    if (!parse_cache(text, key, &entries, &msg)) {
        qrt::set_error(msg);
        return QUBO_EINVAL;
    }
    for (const auto &e : entries) qplan::tune_put(e);
    if (loaded) *loaded = int(entries.size());
    return QUBO_OK;
}

// ------------------------------------------------------------ tuning runs

// Synthetic tuning instance: counter-based SplitMix64 stream (seeded by n),
// int32 entries uniform in [-100, 100] or float32 uniform in [-1, 1).  The
// walk executes the same instructions whatever the values (one add per state;
// the rare candidate path aside), but its speed still moves a few percent
// with them: wider entries toggle more bits per add and the chip holds a
// lower clock (n = 44: 285 ms for [-100, 100] against 301 ms for
// [-10^4, 10^4] on one box).  The ranking of plans is what the sweep keeps,
// and plans of different row caches can swap places within that margin.
uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

std::vector<uint32_t> tuning_instance(int n, qubo_dtype_t dtype)
{
    std::vector<uint32_t> q(size_t(n) * size_t(n));
    for (size_t k = 0; k < q.size(); k++) {
        const uint64_t r = splitmix64((uint64_t(n) << 32) ^ k);
        if (dtype == QUBO_INT32) {
            const int32_t v = int32_t(r % 201) - 100;
            std::memcpy(&q[k], &v, 4);
        } else {
            const float v = float(double(r >> 40) * 0x1.0p-23 - 1.0);
            std::memcpy(&q[k], &v, 4);
        }
    }
    return q;
}

struct Candidate {
    qubo_options_t opt;
    double best_ms = 1e300;
};

// Every plan the library's kernels can run for n: suffix widths, row caches, tiers and
// work-item sizes around the default.
qubo_status_t candidates(const void *Q, int n, qubo_dtype_t dtype, std::vector<Candidate> *out)
{
    static const int kCaches[] = {12, 8, 6, 5, 4, 3};
    for (int B = 6; B <= 10; B++) {
        if (n - B < qplan::kSuper) continue;
        const int mcols = (1 << B) / qplan::kWave;
        for (int G : kCaches) {
            if (!qk::walk_variant_exists(mcols, G)) continue;
            for (int tier = 1; tier <= 2; tier++) {
                qubo_options_t o{};
                o.B = B;
                o.tier = tier;
                o.vgpr_levels = G;
                qplan::Plan P;
                std::string msg;
                qubo_status_t st = qplan::make_plan(Q, n, dtype, &o, &P, &msg);
                if (st != QUBO_OK) {
                    qrt::set_error(msg);
                    return st;
                }
                for (int dL = -2; dL <= 2; dL += 2) {
                    const int L = P.L + dL;
                    if (L < qplan::kSuper || L > P.A || P.A - L > 20) continue;
                    Candidate c;
                    c.opt = o;
                    c.opt.L = L;
                    out->push_back(c);
                }
            }
        }
    }
    return QUBO_OK;
}

qubo_status_t run_candidate(const void *Q, int n, qubo_dtype_t dtype, const qubo_options_t &o,
                            hipStream_t stream, qubo_result_t *r)
{
    qrt::Job job;
    job.plans.resize(1);
    std::string msg;
    qubo_status_t st = qplan::make_plan(Q, n, dtype, &o, &job.plans[0], &msg);
    if (st != QUBO_OK) {
        qrt::set_error(msg);
        return st;
    }
    job.qf.push_back(dtype == QUBO_FP32 ? static_cast<const float *>(Q) : nullptr);
    return qrt::solve_planned(job, stream, 0, r);
}

qubo_status_t tune_one(int n, qubo_dtype_t dtype, int reps, hipStream_t stream,
                       qplan::TuneEntry *winner)
{
    const std::vector<uint32_t> q = tuning_instance(n, dtype);
    std::vector<Candidate> cands;
    qubo_status_t st = candidates(q.data(), n, dtype, &cands);
    if (st != QUBO_OK) return st;
    if (cands.empty()) {
        qrt::set_error("no walk plan for n = " + std::to_string(n));
        return QUBO_EINVAL;
    }
    qubo_result_t ref{}, r{};
    // warm-up (first launches load code objects), and the reference answer
    if ((st = run_candidate(q.data(), n, dtype, cands[0].opt, stream, &ref)) != QUBO_OK) return st;
    auto check = [&](const qubo_result_t &x, const qubo_options_t &o) {
        if (x.best.energy_i == ref.best.energy_i && x.best.index == ref.best.index) return true;
        char buf[200];
        std::snprintf(buf, sizeof(buf),
                      "plan invariance violated at n=%d: B=%d L=%d tier=%d vgpr_levels=%d gave "
                      "(%lld, %llu), expected (%lld, %llu)",
                      n, o.B, o.L, o.tier, o.vgpr_levels, (long long)x.best.energy_i,
                      (unsigned long long)x.best.index, (long long)ref.best.energy_i,
                      (unsigned long long)ref.best.index);
        qrt::set_error(buf);
        return false;
    };
    // pass 1: every candidate once
    for (Candidate &c : cands) {
        if ((st = run_candidate(q.data(), n, dtype, c.opt, stream, &r)) != QUBO_OK) return st;
        if (!check(r, c.opt)) return QUBO_EINTERNAL;
        c.best_ms = r.kernel_ms;
    }
    // pass 2: the four fastest again, keeping each one's minimum
    std::stable_sort(cands.begin(), cands.end(),
                     [](const Candidate &a, const Candidate &b) { return a.best_ms < b.best_ms; });
    const size_t top = std::min<size_t>(4, cands.size());
    for (int rep = 0; rep < reps; rep++)
        for (size_t k = 0; k < top; k++) {
            if ((st = run_candidate(q.data(), n, dtype, cands[k].opt, stream, &r)) != QUBO_OK) return st;
            if (!check(r, cands[k].opt)) return QUBO_EINTERNAL;
            cands[k].best_ms = std::min(cands[k].best_ms, double(r.kernel_ms));
        }
    std::stable_sort(cands.begin(), cands.begin() + long(top),
                     [](const Candidate &a, const Candidate &b) { return a.best_ms < b.best_ms; });
    const Candidate &w = cands[0];
    winner->n = n;
    winner->dtype = dtype;
    winner->B = w.opt.B;
    winner->L = w.opt.L;
    winner->tier = w.opt.tier;
    winner->vgpr_levels = w.opt.vgpr_levels;
    winner->walk_ms = w.best_ms;
    return QUBO_OK;
}

// Batch scope: m copies of the tuning instance of n in one batch, timed by
// a graph replay (2^39 states where 4096 copies reach that: the walk then
// dominates the replay, as it does in real batches).
int batch_copies(int n) { return n >= 39 ? 1 : std::min(4096, 1 << (39 - n)); }

// A batch-scope winner must beat the built-in plan by this margin: every
// extra kernel variant in a batch is one more persistent launch with its own
// tail, which a per-n timing does not see (measured: per-n winners 2-5%
// ahead at n = 20-28 made a mixed 4096-instance batch up to 1% slower).
constexpr double kBatchMargin = 0.95;

qubo_status_t time_batch(const std::vector<const void *> &ptrs, const std::vector<int> &ns,
                         const std::vector<qubo_dtype_t> &dts, const qubo_options_t &o, int runs,
                         double *ms, qubo_result_t *first, qubo_result_t *last)
{
    qubo_batch_t *b = nullptr;
    qubo_status_t st = qubo_batch_create(int(ptrs.size()), ptrs.data(), ns.data(), dts.data(), &o, &b);
    if (st != QUBO_OK) return st;
    *ms = 1e300;
    for (int r = 0; r < runs && st == QUBO_OK; r++) {
        st = qubo_batch_run(b, nullptr);
        double states = 0, kms = 0;
        if (st == QUBO_OK) st = qubo_batch_stats(b, &states, &kms);
        if (st == QUBO_OK && r > 0) *ms = std::min(*ms, kms);   // run 0 warms up
    }
    std::vector<qubo_result_t> res(ptrs.size());
    if (st == QUBO_OK) st = qubo_batch_results(b, res.data());
    if (st == QUBO_OK) {
        *first = res.front();
        *last = res.back();
    }
    const std::string keep = qrt::last_error_cstr();
    qubo_batch_destroy(b);
    qrt::set_error(keep);
    return st;
}

qubo_status_t tune_batch_one(int n, qubo_dtype_t dtype, int reps, qplan::TuneEntry *winner)
{
    const std::vector<uint32_t> q = tuning_instance(n, dtype);
    const int m = batch_copies(n);
    const std::vector<const void *> ptrs(size_t(m), q.data());
    const std::vector<int> ns(size_t(m), n);
    const std::vector<qubo_dtype_t> dts(size_t(m), dtype);
    // (B, row cache, tier) as for a lone solve; L stays the batch default
    std::vector<Candidate> cands, all;
    qubo_status_t st = candidates(q.data(), n, dtype, &all);
    if (st != QUBO_OK) return st;
    for (const Candidate &c : all) {
        bool dup = false;
        for (const Candidate &d : cands)
            dup |= d.opt.B == c.opt.B && d.opt.tier == c.opt.tier && d.opt.vgpr_levels == c.opt.vgpr_levels;
        if (dup) continue;
        Candidate k = c;
        k.opt.L = 0;
        cands.push_back(k);
    }
    if (cands.empty()) {
        qrt::set_error("no walk plan for n = " + std::to_string(n));
        return QUBO_EINVAL;
    }
    qubo_result_t ref{}, r0{}, r1{};
    bool have_ref = false;
    auto check = [&](const qubo_options_t &o) {
        if (!have_ref) {
            ref = r0;
            have_ref = true;
        }
        for (const qubo_result_t *x : {&r0, &r1})
            if (x->best.energy_i != ref.best.energy_i || x->best.index != ref.best.index) {
                char buf[200];
                std::snprintf(buf, sizeof(buf),
                              "plan invariance violated in a batch at n=%d: B=%d tier=%d "
                              "vgpr_levels=%d gave (%lld, %llu), expected (%lld, %llu)",
                              n, o.B, o.tier, o.vgpr_levels, (long long)x->best.energy_i,
                              (unsigned long long)x->best.index, (long long)ref.best.energy_i,
                              (unsigned long long)ref.best.index);
                qrt::set_error(buf);
                return false;
            }
        return true;
    };
    for (Candidate &c : cands) {
        double ms = 0;
        if ((st = time_batch(ptrs, ns, dts, c.opt, 2, &ms, &r0, &r1)) != QUBO_OK) return st;
        if (!check(c.opt)) return QUBO_EINTERNAL;
        c.best_ms = ms;
    }
    std::stable_sort(cands.begin(), cands.end(),
                     [](const Candidate &a, const Candidate &b) { return a.best_ms < b.best_ms; });
    const size_t top = std::min<size_t>(4, cands.size());
    if (reps > 0)
        for (size_t k = 0; k < top; k++) {
            double ms = 0;
            if ((st = time_batch(ptrs, ns, dts, cands[k].opt, reps + 1, &ms, &r0, &r1)) != QUBO_OK)
                return st;
            if (!check(cands[k].opt)) return QUBO_EINTERNAL;
            cands[k].best_ms = std::min(cands[k].best_ms, ms);
        }
    std::stable_sort(cands.begin(), cands.begin() + long(top),
                     [](const Candidate &a, const Candidate &b) { return a.best_ms < b.best_ms; });
    const Candidate *wp = &cands[0];
    // the built-in plan (tier 2 given explicitly: the table is bypassed)
    qplan::Plan D;
    std::string msg;
    qubo_options_t dopt{};
    dopt.tier = 2;
    if (qplan::make_plan(q.data(), n, dtype, &dopt, &D, &msg, true) == QUBO_OK && !D.direct)
        for (const Candidate &c : cands)
            if (c.opt.B == D.B && c.opt.tier == D.tier && c.opt.vgpr_levels == D.vgpr_levels &&
                wp->best_ms >= kBatchMargin * c.best_ms)
                wp = &c;
    const Candidate &w = *wp;
    winner->n = n;
    winner->dtype = dtype;
    winner->B = w.opt.B;
    winner->L = 0;
    winner->tier = w.opt.tier;
    winner->vgpr_levels = w.opt.vgpr_levels;
    winner->walk_ms = w.best_ms;
    winner->scope = qplan::kScopeBatch;
    return QUBO_OK;
}

void to_abi(const qplan::TuneEntry &e, qubo_tune_entry_t *o)
{
    o->n = e.n;
    o->dtype = e.dtype;
    o->B = e.B;
    o->L = e.L;
    o->tier = e.tier;
    o->vgpr_levels = e.vgpr_levels;
    o->walk_ms = e.walk_ms;
    o->scope = e.scope;
}

std::once_flag g_autoload_once;

}  // namespace

namespace qrt {

void tune_autoload()
{
    std::call_once(g_autoload_once, [] {
        const char *path = std::getenv("QUBO_TUNE_CACHE");
        if (!path || !*path) return;
        std::string key;
        if (current_device_key(&key) != QUBO_OK) return;
        const std::string saved = last_error_cstr();
        int loaded = 0;
        if (load_into_table(path, key, &loaded) != QUBO_OK)
            std::fprintf(stderr, "qubo: ignoring QUBO_TUNE_CACHE=%s: %s\n", path, last_error_cstr());
        set_error(saved);
    });
}

}  // namespace qrt

extern "C" {

qubo_status_t qubo_device_key(char *buf, int cap)
{
    try {
        qrt::set_error("");
        if (!buf || cap < 1) {
            qrt::set_error("null buffer");
            return QUBO_EINVAL;
        }
        std::string key;
        qubo_status_t st = current_device_key(&key);
        if (st != QUBO_OK) return st;
        if (int(key.size()) >= cap) {
            qrt::set_error("buffer too small for the device key");
            return QUBO_EINVAL;
        }
        std::memcpy(buf, key.c_str(), key.size() + 1);
        return QUBO_OK;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

qubo_status_t qubo_tune_set(const qubo_tune_entry_t *entries, int count)
{
    try {
        qrt::set_error("");
        if (count < 0 || (count > 0 && !entries)) {
            qrt::set_error("bad entries");
            return QUBO_EINVAL;
        }
        std::vector<qplan::TuneEntry> v(static_cast<size_t>(count));
        for (int k = 0; k < count; k++) {
            qplan::TuneEntry &e = v[size_t(k)];
            e.n = entries[k].n;
            e.dtype = entries[k].dtype;
            e.B = entries[k].B;
            e.L = entries[k].L;
            e.tier = entries[k].tier;
            e.vgpr_levels = entries[k].vgpr_levels;
            e.walk_ms = entries[k].walk_ms;
            e.scope = entries[k].scope;
            std::string msg;
            if (!qplan::tune_valid(e, &msg)) {
                qrt::set_error("entry " + std::to_string(k) + ": " + msg);
                return QUBO_EINVAL;
            }
        }
        for (const auto &e : v) qplan::tune_put(e);
        return QUBO_OK;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

int qubo_tune_lookup(int n, qubo_dtype_t dtype, int scope, qubo_tune_entry_t *out)
{
    qplan::TuneEntry e;
    if (!qplan::tune_get(n, dtype, scope, &e)) return 0;
    if (out) to_abi(e, out);
    return 1;
}

void qubo_tune_clear(void) { qplan::tune_clear(); }

qubo_status_t qubo_tune_load(const char *path, const char *device_key, int *loaded)
{
    try {
        qrt::set_error("");
        if (!path) {
            qrt::set_error("null path");
            return QUBO_EINVAL;
        }
        std::string key;
        if (device_key) {
            key = device_key;
        } else {
            qubo_status_t st = current_device_key(&key);
            if (st != QUBO_OK) return st;
        }
        return load_into_table(path, key, loaded);
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

qubo_status_t qubo_tune_save(const char *path, const char *device_key)
{
    try {
        qrt::set_error("");
        if (!path) {
            qrt::set_error("null path");
            return QUBO_EINVAL;
        }
        std::string key;
        if (device_key) {
            key = device_key;
        } else {
            qubo_status_t st = current_device_key(&key);
            if (st != QUBO_OK) return st;
        }
        if (key.find('"') != std::string::npos || key.find('\\') != std::string::npos) {
            qrt::set_error("device key may not contain quotes or backslashes");
            return QUBO_EINVAL;
        }
        std::string msg;
        if (!write_file(path, format_cache(qplan::tune_all(), key), &msg)) {
            qrt::set_error(msg);
            return QUBO_EINVAL;
        }
        return QUBO_OK;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

}  // extern "C"

namespace {

qubo_status_t autotune_range(bool batch, int n_min, int n_max, qubo_dtype_t dtype, int reps,
                             const char *cache_path, qubo_tune_entry_t *out, int out_cap,
                             int *out_count)
{
    const int hi = batch ? 44 : 48;
    if (n_min < qplan::kDirectMaxN + 1 || n_max > hi || n_min > n_max) {
        qrt::set_error("autotune range must satisfy 15 <= n_min <= n_max <= " + std::to_string(hi));
        return QUBO_EINVAL;
    }
    if (dtype != QUBO_INT32 && dtype != QUBO_FP32) {
        qrt::set_error("unknown dtype");
        return QUBO_EINVAL;
    }
    if (reps < 0 || reps > 100 || out_cap < 0 || (out_cap > 0 && !out)) {
        qrt::set_error("bad reps or output buffer");
        return QUBO_EINVAL;
    }
    qubo_status_t st;
    hipStream_t stream = qrt::thread_stream(&st);
    if (st != QUBO_OK) return st;
    std::string key;
    if ((st = current_device_key(&key)) != QUBO_OK) return st;
    std::vector<qplan::TuneEntry> won;
    for (int n = n_min; n <= n_max; n++) {
        qplan::TuneEntry e;
        st = batch ? tune_batch_one(n, dtype, reps, &e) : tune_one(n, dtype, reps, stream, &e);
        if (st != QUBO_OK) return st;
        won.push_back(e);
    }
    if (cache_path) {
        // merge with what the file already holds for this device
        std::string text, msg;
        if (read_file(cache_path, &text, &msg)) {
            std::vector<qplan::TuneEntry> old;
            if (parse_cache(text, key, &old, &msg))
                for (const auto &e : old) qplan::tune_put(e);
        }
    }
    for (const auto &e : won) qplan::tune_put(e);
    if (cache_path) {
        std::string msg;
        if (!write_file(cache_path, format_cache(qplan::tune_all(), key), &msg)) {
            qrt::set_error(msg);
            return QUBO_EINVAL;
        }
    }
    for (int k = 0; k < out_cap && k < int(won.size()); k++) to_abi(won[size_t(k)], &out[k]);
    if (out_count) *out_count = int(won.size());
    return QUBO_OK;
}

}  // namespace

extern "C" {

qubo_status_t qubo_autotune(int n_min, int n_max, qubo_dtype_t dtype, int reps,
                            const char *cache_path, qubo_tune_entry_t *out, int out_cap,
                            int *out_count)
{
    try {
        qrt::set_error("");
        return autotune_range(false, n_min, n_max, dtype, reps, cache_path, out, out_cap, out_count);
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

qubo_status_t qubo_autotune_batch(int n_min, int n_max, qubo_dtype_t dtype, int reps,
                                  const char *cache_path, qubo_tune_entry_t *out, int out_cap,
                                  int *out_count)
{
    try {
        qrt::set_error("");
        return autotune_range(true, n_min, n_max, dtype, reps, cache_path, out, out_cap, out_count);
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

}  // extern "C"

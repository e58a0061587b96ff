// host_checks.cpp -- host-only checks of the library's planner, file formats
// and serving policy, built with g++ under AddressSanitizer and
// UndefinedBehaviorSanitizer (and ThreadSanitizer for the oracle's threads)
// by tests/test_host_sanitized.py.  TEST CODE: the mock device below finishes
// requests with the CPU oracle; it is a test double, never a product path.
//
//   host_checks plan    -- make_plan over n = 1..60, int32 and float32 inputs,
//                          including the int32 exactness edge and non-finite
//                          entries; checks the plan's invariants
//   host_checks json    -- tuning-cache round trip and 20000 mutated texts
//   host_checks ckpt    -- checkpoint round trip and 4000 mutated files
//   host_checks sched   -- the serving policy driven by a mock queue and
//                          device; every request's result is the oracle's
//   host_checks oracle  -- the oracle's threaded entry points (TSan build)
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "hostio.h"
#include "plan.h"
#include "serve_policy.h"

extern "C" {
int oracle_solve_i(int n, const int32_t *Q, uint64_t first, uint64_t count, int k, int threads,
                   int64_t *E, uint64_t *idx);
int oracle_gray_i(int n, const int32_t *Q, int threads, int64_t *E, uint64_t *idx);
}

static int g_fail = 0;
#define CHECK(cond)                                                                \
    do {                                                                           \
        if (!(cond)) {                                                             \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            if (++g_fail > 20) std::exit(1);                                       \
        }                                                                          \
    } while (0)

// ---------------------------------------------------------------- plan
static int run_plan()
{
    std::mt19937_64 rng(1);
    int plans = 0;
    for (int n = 1; n <= 60; n++) {
        for (int kind = 0; kind < 5; kind++) {
            std::vector<int32_t> qi(size_t(n) * n, 0);
            std::vector<float> qf(size_t(n) * n, 0.f);
            const bool fp = kind >= 3;
            int64_t lo = kind == 0 ? -100 : (kind == 1 ? -10000 : 0);
            for (int i = 0; i < n; i++)
                for (int j = 0; j < n; j++) {
                    if (kind == 2) {   // spread 2^30 - 1 over the upper triangle
                        continue;
                    }
                    if (!fp && (kind == 0 || kind == 1))
                        qi[size_t(i) * n + j] = int32_t(int64_t(rng() % uint64_t(2 * -lo + 1)) + lo);
                    if (fp) qf[size_t(i) * n + j] = float(std::ldexp(double(int64_t(rng() % 2001) - 1000), -7));
                }
            if (kind == 2) {   // the int32 exactness edge: sum |T| = 2^30 - 1, then one more
                const int64_t total = (int64_t(1) << 30) - 1;
                const int64_t m = int64_t(n) * (n + 1) / 2;
                int64_t left = total;
                for (int i = 0; i < n; i++)
                    for (int j = i; j < n; j++) {
                        const int64_t v = (i == n - 1 && j == n - 1) ? left : total / m;
                        qi[size_t(i) * n + j] = int32_t((i + j) % 2 ? -v : v);
                        left -= v;
                    }
            }
            if (kind == 4 && n > 2) qf[size_t(1) * n + 2] = std::numeric_limits<float>::infinity();
            qplan::Plan P;
            std::string msg;
            const qubo_status_t st = qplan::make_plan(fp ? static_cast<const void *>(qf.data())
                                                         : static_cast<const void *>(qi.data()),
                                                      n, fp ? QUBO_FP32 : QUBO_INT32, nullptr, &P, &msg);
            if (kind == 4 && n > 2) {
                CHECK(st == QUBO_ENONFINITE);
                continue;
            }
            CHECK(st == QUBO_OK);
            if (st != QUBO_OK) continue;
            plans++;
            CHECK(P.n == n && int(P.T.size()) == n * n);
            CHECK(P.sum_abs <= qplan::kIntSumLimit);
            for (int i = 0; i < n; i++)
                for (int j = 0; j < i; j++) CHECK(P.T[size_t(i) * n + j] == 0);
            if (P.direct) {
                CHECK(n <= qplan::kDirectMaxN);
            } else {
                CHECK(P.A + P.B == n && P.B >= 6 && P.B <= (P.tier == 4 ? 11 : 10) && P.L >= 6 &&
                      P.L <= P.A);
                CHECK(P.items == (uint64_t(1) << (P.A - P.L)));
                // the packed tier only where every chunk energy fits 16 bits
                int32_t c = 0;
                if (P.tier == 4) {
                    CHECK(!fp && P.B >= 9 && qplan::packed_shift(P, P.A, &c) && c == P.pack_shift);
                    int64_t lo = 0, hi = 0;
                    qplan::chunk_energy_range(P, P.A, &lo, &hi);
                    CHECK(lo + c >= -32768 && hi + c <= 32767);
                    CHECK(P.sum_abs + (c < 0 ? -int64_t(c) : int64_t(c)) <= qplan::kIntSumLimit);
                } else {
                    CHECK(fp || P.B < 8 || P.A - 1 < qplan::kSuper || !qplan::packed_shift(P, P.A - 1, &c));
                    // the int32 walk's chunk energies start at 0 (or no shift
                    // where the int32 bound would not hold it)
                    int64_t lo = 0, hi = 0;
                    qplan::chunk_energy_range(P, P.A, &lo, &hi);
                    const int64_t a = lo < 0 ? -lo : lo;
                    CHECK(P.pack_shift == (P.sum_abs + a <= qplan::kIntSumLimit ? -lo : 0));
                }
            }
            if (kind == 2) {   // one more unit of |T| is refused
                int32_t &e = qi[size_t(n - 1) * n + (n - 1)];
                e += e >= 0 ? 1 : -1;
                qplan::Plan P2;
                CHECK(qplan::make_plan(qi.data(), n, QUBO_INT32, nullptr, &P2, &msg) == QUBO_EOVERFLOW);
            }
            if (fp) CHECK(P.eps_q >= 0.0 && P.p >= 0);
        }
    }
    qplan::Plan P;
    std::string msg;
    CHECK(qplan::make_plan(nullptr, 10, QUBO_INT32, nullptr, &P, &msg) != QUBO_OK);
    int32_t one = 5;
    CHECK(qplan::make_plan(&one, 0, QUBO_INT32, nullptr, &P, &msg) == QUBO_EINVAL);
    CHECK(qplan::make_plan(&one, 61, QUBO_INT32, nullptr, &P, &msg) == QUBO_EINVAL);
    std::printf("plan: %d plans checked\n", plans);
    return g_fail ? 1 : 0;
}

// ---------------------------------------------------------------- mutations
static std::string mutate(const std::string &s, std::mt19937_64 &rng)
{
    std::string m = s;
    const int kind = int(rng() % 6);
    const size_t at = m.empty() ? 0 : size_t(rng() % m.size());
    static const char junk[] = "{}[]\":,0123456789.-+eE \n\\tfnrux\x01\xff";
    switch (kind) {
    case 0: if (!m.empty()) m[at] = junk[rng() % (sizeof junk - 1)]; break;
    case 1: m.resize(at); break;
    case 2: m.insert(at, 1, junk[rng() % (sizeof junk - 1)]); break;
    case 3: if (!m.empty()) m.erase(at, 1 + rng() % 8); break;
    case 4: m.insert(at, std::string(1 + rng() % 200, junk[rng() % (sizeof junk - 1)])); break;
    default: for (int r = 0; r < 4 && !m.empty(); r++) m[rng() % m.size()] ^= char(1 << (rng() % 8)); break;
    }
    return m;
}

// ---------------------------------------------------------------- json
static int run_json()
{
    std::vector<qplan::TuneEntry> in;
    for (int n = 16; n <= 44; n++) {   // n - B must hold one 64-step super-block
        qplan::TuneEntry e;
        e.n = n;
        e.dtype = n % 3 ? QUBO_INT32 : QUBO_FP32;
        e.B = 10;
        e.L = 0;
        e.tier = 1 + n % 2;
        e.vgpr_levels = (n % 4 == 0) ? 12 : 4;
        e.walk_ms = 0.125 * n;
        e.scope = n % 5 ? qplan::kScopeSingle : qplan::kScopeBatch;
        std::string why;
        CHECK(qplan::tune_valid(e, &why));
        in.push_back(e);
    }
    const std::string text = qhost::format_cache(in, "gfx950/256cu");
    std::vector<qplan::TuneEntry> out;
    std::string msg;
    CHECK(qhost::parse_cache(text, "gfx950/256cu", &out, &msg));
    CHECK(out.size() == in.size());
    for (size_t k = 0; k < out.size() && k < in.size(); k++)
        CHECK(out[k].n == in[k].n && out[k].dtype == in[k].dtype && out[k].B == in[k].B &&
              out[k].L == in[k].L && out[k].tier == in[k].tier &&
              out[k].vgpr_levels == in[k].vgpr_levels && out[k].walk_ms == in[k].walk_ms &&
              out[k].scope == in[k].scope);
    out.clear();
    CHECK(!qhost::parse_cache(text, "gfx942/304cu", &out, &msg));
    std::mt19937_64 rng(2);
    int ok = 0;
    for (int it = 0; it < 20000; it++) {
        std::string m = mutate(text, rng);
        if (it % 3 == 0) m = mutate(m, rng);
        std::vector<qplan::TuneEntry> got;
        std::string why;
        if (qhost::parse_cache(m, "gfx950/256cu", &got, &why)) {
            ok++;
            for (const auto &e : got) {
                std::string w2;
                CHECK(qplan::tune_valid(e, &w2));
            }
        } else {
            CHECK(!why.empty());
        }
    }
    // deep nesting and huge inputs are refused, not recursed into
    std::string deep(100000, '[');
    std::vector<qplan::TuneEntry> got;
    CHECK(!qhost::parse_cache(deep, "gfx950/256cu", &got, &msg));
    std::printf("json: round trip ok, %d of 20000 mutated texts still valid\n", ok);
    return g_fail ? 1 : 0;
}

// ---------------------------------------------------------------- ckpt
static int run_ckpt(const char *dir)
{
    const std::string path = std::string(dir) + "/c.ckpt";
    qhost::Ckpt c;
    c.n = 40;
    c.dtype = QUBO_INT32;
    c.qhash = 0x0123456789abcdefull;
    c.A = 30;
    c.B = 10;
    c.L = 14;
    c.tier = 2;
    c.vgpr_levels = 4;
    c.items = 65536;
    c.next_item = 4096;
    c.found = 1;
    c.energy_i = -12345;
    c.energy = -12345.0;
    c.index = 987654321;
    c.walk_ms = 12.5;
    std::string msg;
    CHECK(qhost::write_ckpt(path.c_str(), c, &msg));
    qhost::Ckpt r;
    CHECK(qhost::read_ckpt(path.c_str(), &r, &msg) == 1);
    CHECK(r.n == c.n && r.qhash == c.qhash && r.items == c.items && r.next_item == c.next_item &&
          r.energy_i == c.energy_i && r.index == c.index && r.walk_ms == c.walk_ms);
    CHECK(qhost::read_ckpt((std::string(dir) + "/missing.ckpt").c_str(), &r, &msg) == 0);
    FILE *f = std::fopen(path.c_str(), "rb");
    std::string text;
    for (int ch; (ch = std::fgetc(f)) != EOF;) text.push_back(char(ch));
    std::fclose(f);
    std::mt19937_64 rng(3);
    int ok = 0;
    const std::string mpath = std::string(dir) + "/m.ckpt";
    for (int it = 0; it < 4000; it++) {
        const std::string m = mutate(text, rng);
        FILE *g = std::fopen(mpath.c_str(), "wb");
        std::fwrite(m.data(), 1, m.size(), g);
        std::fclose(g);
        qhost::Ckpt x;
        std::string why;
        const int rc = qhost::read_ckpt(mpath.c_str(), &x, &why);
        CHECK(rc == 1 || rc == -1);
        if (rc == 1) {
            ok++;
            CHECK(x.n >= 1 && x.n <= qplan::kMaxN && x.next_item <= x.items);
            CHECK(x.index < (uint64_t(1) << x.n));
        }
    }
    std::printf("ckpt: round trip ok, %d of 4000 mutated files still valid\n", ok);
    return g_fail ? 1 : 0;
}

// ---------------------------------------------------------------- sched
// The serving policy (qsched) driven by a mock queue and a mock device: a
// tick admits requests, hands out item shares, "runs" them, and finishes
// each request whose items are all issued by asking the CPU oracle for its
// answer.  The checks: memory and slots stay within their limits,
// admission is first come first served and is deferred when memory is
// short, slots are recycled, every admitted request finishes, and every
// ticket's result is the oracle's answer for its own matrix.
struct MockReq {
    uint64_t ticket = 0;
    int n = 0;
    std::vector<int32_t> Q;
    size_t bytes = 0;
    uint64_t items = 0, next = 0;
    int slot = -1;
    int arrival = 0;
};

static int run_sched()
{
    std::mt19937_64 rng(4);
    const size_t budget = 3u << 20;
    const int max_slots = 6;
    const uint64_t tick_items = 16;
    std::vector<MockReq> reqs;
    int rejected = 0;
    for (int k = 0; k < 160; k++) {
        MockReq r;
        r.ticket = uint64_t(k) + 1;
        r.n = 8 + int(rng() % 11);                       // 8..18
        r.Q.resize(size_t(r.n) * r.n, 0);
        for (int i = 0; i < r.n; i++)
            for (int j = i; j < r.n; j++) r.Q[size_t(i) * r.n + j] = int32_t(int64_t(rng() % 201) - 100);
        r.items = (r.n <= 14) ? 0 : (uint64_t(1) << (r.n - 12));   // direct plans have no items
        r.bytes = size_t(64 + r.n * r.n * 4 + r.items * 16) * 1024;
        if (k % 37 == 36) r.bytes = budget + 1;            // can never fit: refused at submit
        r.arrival = k / 3;                                 // three arrivals per tick
        reqs.push_back(std::move(r));
    }
    std::deque<size_t> queue;
    std::vector<size_t> active;
    std::vector<int> free_slots;
    for (int s = max_slots - 1; s >= 0; s--) free_slots.push_back(s);
    size_t mem = 0, next_arrival = 0;
    uint64_t last_admitted = 0;
    int deferrals = 0, slot_uses = 0, finished = 0;
    std::map<uint64_t, std::pair<int64_t, uint64_t>> results;   // ticket -> (E, index)
    for (int tick = 0; tick < 100000 && (finished + rejected < int(reqs.size())); tick++) {
        while (next_arrival < reqs.size() && reqs[next_arrival].arrival <= tick) {
            if (reqs[next_arrival].bytes > budget) rejected++;   // submit refuses it
            else queue.push_back(next_arrival);
            next_arrival++;
        }
        std::vector<size_t> qbytes;
        for (size_t i : queue) qbytes.push_back(reqs[i].bytes);
        const size_t nfree = std::min(size_t(max_slots) - active.size(), free_slots.size());
        const size_t n_adm = qsched::admit_count(qbytes, mem, budget, nfree);
        CHECK(n_adm <= queue.size() && n_adm <= nfree);
        if (n_adm < queue.size() && n_adm < nfree) deferrals++;   // memory, not slots, held one back
        for (size_t a = 0; a < n_adm; a++) {
            MockReq &r = reqs[queue.front()];
            queue.pop_front();
            CHECK(r.ticket > last_admitted);                        // first come, first served
            last_admitted = r.ticket;
            mem += r.bytes;
            r.slot = free_slots.back();
            free_slots.pop_back();
            slot_uses++;
            active.push_back(size_t(&r - reqs.data()));
        }
        CHECK(mem <= budget && int(active.size()) <= max_slots);
        // one tick of work: water-filled shares, fewest remaining first
        std::vector<size_t> walkers;
        for (size_t i : active)
            if (reqs[i].next < reqs[i].items) walkers.push_back(i);
        std::sort(walkers.begin(), walkers.end(), [&](size_t a, size_t b) {
            return reqs[a].items - reqs[a].next < reqs[b].items - reqs[b].next;
        });
        std::vector<uint64_t> left;
        for (size_t i : walkers) left.push_back(reqs[i].items - reqs[i].next);
        const std::vector<uint64_t> share = qsched::tick_shares(left, tick_items);
        uint64_t sum = 0, backlog = 0;
        for (size_t k = 0; k < walkers.size(); k++) {
            CHECK(share[k] >= 1 && share[k] <= left[k]);
            reqs[walkers[k]].next += share[k];
            sum += share[k];
            backlog += left[k];
        }
        if (!walkers.empty())
            CHECK(sum <= std::max<uint64_t>(qsched::tick_scale(backlog, tick_items) * tick_items,
                                            walkers.size()));
        // finish: every request whose items are all issued (direct ones at once)
        for (size_t a = 0; a < active.size();) {
            MockReq &r = reqs[active[a]];
            if (r.next < r.items) {
                a++;
                continue;
            }
            int64_t E = 0;
            uint64_t idx = 0;
            CHECK(oracle_solve_i(r.n, r.Q.data(), 0, uint64_t(1) << r.n, 1, 1, &E, &idx) == 0);
            CHECK(results.count(r.ticket) == 0);
            results[r.ticket] = {E, idx};
            mem -= r.bytes;
            free_slots.push_back(r.slot);
            finished++;
            active.erase(active.begin() + long(a));
        }
    }
    CHECK(finished + rejected == int(reqs.size()));
    CHECK(mem == 0 && active.empty() && queue.empty());
    CHECK(deferrals > 0);                    // the budget held admission back at least once
    CHECK(slot_uses > max_slots);            // slots were recycled
    CHECK(rejected == int(reqs.size()) / 37);
    // each ticket's answer is the oracle's for its own matrix (a second,
    // independent evaluation: the Gray-walk form)
    for (const MockReq &r : reqs) {
        if (r.bytes > budget) {
            CHECK(results.count(r.ticket) == 0);
            continue;
        }
        auto it = results.find(r.ticket);
        CHECK(it != results.end());
        if (it == results.end()) continue;
        int64_t E = 0;
        uint64_t idx = 0;
        CHECK(oracle_gray_i(r.n, r.Q.data(), 1, &E, &idx) == 0);
        CHECK(it->second.first == E && it->second.second == idx);
    }
    // policy edge cases
    CHECK(qsched::admit_count({}, 0, 100, 4) == 0);
    CHECK(qsched::admit_count({10, 10, 10}, 0, 100, 0) == 0);
    CHECK(qsched::admit_count({60, 10, 30}, 0, 100, 8) == 3);
    CHECK(qsched::admit_count({60, 50, 1}, 0, 100, 8) == 1);          // no overtaking
    CHECK(qsched::admit_count({size_t(-1)}, 0, 100, 8) == 0);         // no overflow
    CHECK(qsched::tick_shares({}, 8).empty());
    CHECK(qsched::tick_shares({1, 100}, 8) == std::vector<uint64_t>({1, 31}));   // backlog 101: scale 4
    CHECK(qsched::tick_scale(0, 8) == 1 && qsched::tick_scale(1u << 20, 8) == qsched::kMaxTickScale);
    CHECK(qsched::tick_scale(4 * 16 * 8, 8) == 16 && qsched::tick_scale(4 * 16 * 8 + 1, 8) == 32);
    std::printf("sched: %d finished, %d refused, %d deferrals, %d slot uses\n", finished, rejected,
                deferrals, slot_uses);
    return g_fail ? 1 : 0;
}

// ---------------------------------------------------------------- oracle threads
static int run_oracle()
{
    std::mt19937_64 rng(5);
    for (int n : {12, 17, 20}) {
        std::vector<int32_t> Q(size_t(n) * n, 0);
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) Q[size_t(i) * n + j] = int32_t(int64_t(rng() % 401) - 200);
        int64_t E1[8], E2 = 0;
        uint64_t I1[8], I2 = 0;
        CHECK(oracle_solve_i(n, Q.data(), 0, uint64_t(1) << n, 8, 6, E1, I1) == 0);
        CHECK(oracle_gray_i(n, Q.data(), 5, &E2, &I2) == 0);
        CHECK(E1[0] == E2 && I1[0] == I2);
        for (int k = 1; k < 8; k++) CHECK(E1[k] > E1[k - 1] || (E1[k] == E1[k - 1] && I1[k] > I1[k - 1]));
    }
    std::printf("oracle: threaded O1 and O2 agree\n");
    return g_fail ? 1 : 0;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    const std::string what = argv[1];
    if (what == "plan") return run_plan();
    if (what == "json") return run_json();
    if (what == "ckpt") return run_ckpt(argc > 2 ? argv[2] : ".");
    if (what == "sched") return run_sched();
    if (what == "oracle") return run_oracle();
    return 2;
}

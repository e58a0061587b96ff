// server.cpp -- continuous-batching solve server.
//
// Requests are planned on the submitting thread and queued.  One scheduler
// thread owns the device stream and runs ticks:
//   1. admission: queued requests enter device slots, first come first
//      served, while a slot is free and the device-memory budget allows;
//      each admitted request gets one allocation (its tables, per-item
//      results) and a table-build launch; the tables stay resident until it
//      finishes;
//   2. one persistent walk launch over a slice of work items from EVERY
//      admitted request (water-filling: requests with few items left get all
//      of them, the rest share the remaining per-tick item budget), so a
//      request arriving while others are on the GPU joins the next tick;
//   3. a finish launch for requests whose last items ran in this tick, and
//      one small result download.
// Ticks alternate between two buffer sets: tick k+1 is enqueued before the
// host waits for tick k, so the GPU does not idle between ticks.  A request
// is solved by the same kernels and the same integer arithmetic whether it
// runs alone or mixed with others, so its result does not depend on the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "runtime.h"
#include "serve_policy.h"

namespace {

using Clock = std::chrono::steady_clock;

// Walk launches per tick are one per distinct walk kernel variant among the
// active requests; this bounds the number of built variants (B x cache x tier).
constexpr int kMaxTickLaunches = 32;
constexpr int kServeL = 12;         // log2 Gray steps per work item of a served request

enum class RState { Queued, Active, Done, Failed };

struct Request {
    uint64_t ticket = 0;
    qrt::Job job;                 // single-instance job
    std::vector<float> qf;        // owned float32 input
    Clock::time_point arrival;
    RState state = RState::Queued;
    void *d_mem = nullptr;
    int kslot = -1;
    qk::Inst base{};              // device descriptor of the whole instance
    uint64_t next_item = 0;       // next work item to issue
    qubo_result_t result{};
    qubo_status_t status = QUBO_OK;
    std::string error;
};

struct TickBuf {
    hipEvent_t done = nullptr;
    qk::Inst *h_walk = nullptr, *d_walk = nullptr;   // walk descriptors (max_slots)
    qk::Inst *h_fin = nullptr, *d_fin = nullptr;     // finish descriptors (max_slots)
    qk::FinalRes *h_out = nullptr, *d_out = nullptr; // finish results (max_slots)
    std::vector<Request *> finishing;
    bool inflight = false;
};

}  // namespace

struct qubo_server {
    int dev = 0;
    size_t budget = 0;
    int max_slots = 0;
    int cus = 0;                  // compute units of the device
    uint64_t tick_items = 0;      // work items per tick (two per resident wave)
    hipStream_t stream = nullptr;
    int32_t *d_karena = nullptr;  // max_slots K tables
    qk::Inst *d_setup = nullptr;  // descriptors of the requests admitted in one round
    unsigned long long *d_counter = nullptr;
    std::vector<int> free_kslots;
    TickBuf ticks[2];
    int cur = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::unordered_map<uint64_t, Request *> reqs;
    uint64_t next_ticket = 1;
    size_t mem_used = 0, mem_peak = 0;
    int active_peak = 0;
    uint64_t n_ticks = 0;
    bool stop = false;
    std::string fatal;
    std::vector<double> lat_ms;
    double states_done = 0.0;
    bool have_t0 = false;
    Clock::time_point t0;
    std::thread th;
};

namespace {

double ms_since(Clock::time_point a) { return std::chrono::duration<double, std::milli>(Clock::now() - a).count(); }

void fail_all(qubo_server *s, const std::string &msg)
{
    std::lock_guard<std::mutex> lk(s->mu);
    s->fatal = msg;
    for (auto &kv : s->reqs) {
        Request *r = kv.second;
        if (r->state == RState::Queued || r->state == RState::Active) {
            r->state = RState::Failed;
            r->status = QUBO_EDEVICE;
            r->error = msg;
        }
    }
    s->queue.clear();
    s->active.clear();
    s->cv_done.notify_all();
}

// Called with the tick's event complete: publish results, release memory.
void complete_tick(qubo_server *s, TickBuf &t)
{
    std::vector<Request *> done = std::move(t.finishing);
    t.finishing.clear();
    t.inflight = false;
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t i = 0; i < done.size(); i++) {
        Request *r = done[i];
        qubo_status_t st = qrt::job_result(r->job, 0, t.h_out[i], &r->result);
        const double lat = ms_since(r->arrival);
        if (st != QUBO_OK) {
            r->status = st;
            r->error = qrt::last_error_cstr();
            r->state = RState::Failed;
        } else {
            r->result.total_ms = lat;
            r->result.kernel_ms = 0.0;
            r->state = RState::Done;
        }
        s->lat_ms.push_back(lat);
        s->states_done += std::ldexp(1.0, r->job.plans[0].n);
        (void)hipFreeAsync(r->d_mem, s->stream);
        r->d_mem = nullptr;
        s->mem_used -= r->job.bytes;
        s->free_kslots.push_back(r->kslot);
        s->active.erase(std::find(s->active.begin(), s->active.end(), r));
    }
    s->cv_done.notify_all();
}

// Admit queued requests (policy: qsched::admit_count); returns the newly
// admitted ones (device set-up pending).
std::vector<Request *> take_admissions(qubo_server *s)
{
    std::vector<Request *> adm;
    std::vector<size_t> bytes;
    bytes.reserve(s->queue.size());
    for (const Request *r : s->queue) bytes.push_back(r->job.bytes);
    const size_t free_slots = std::min(size_t(s->max_slots) - std::min(size_t(s->max_slots),
                                                                      s->active.size()),
                                       s->free_kslots.size());
    size_t n_adm = qsched::admit_count(bytes, s->mem_used, s->budget, free_slots);
    for (; n_adm > 0; n_adm--) {
        Request *r = s->queue.front();
        s->queue.pop_front();
        s->mem_used += r->job.bytes;
        s->mem_peak = std::max(s->mem_peak, s->mem_used);
        r->kslot = s->free_kslots.back();
        s->free_kslots.pop_back();
        r->state = RState::Active;
        s->active.push_back(r);
        s->active_peak = std::max(s->active_peak, int(s->active.size()));
        adm.push_back(r);
    }
    return adm;
}

qubo_status_t setup_request(qubo_server *s, Request *r)
{
    QRT_HIP(hipMallocAsync(&r->d_mem, r->job.bytes, s->stream), "hipMallocAsync");
    qubo_status_t st = qrt::job_bind(&r->job, r->d_mem);
    if (st != QUBO_OK) return st;
    // The K table lives in the server's arena so one walk launch sees every
    // request's table in a single array.
    qk::Inst I;
    std::memcpy(&I, r->job.stage.data(), sizeof(I));
    I.K = s->d_karena + size_t(r->kslot) * qk::kKTable;
    I.kslot = r->kslot;
    std::memcpy(r->job.stage.data(), &I, sizeof(I));
    r->base = I;
    QRT_HIP(hipMemcpyAsync(r->d_mem, r->job.stage.data(), r->job.stage_bytes, hipMemcpyHostToDevice,
                           s->stream),
            "hipMemcpyAsync H2D");
    return QUBO_OK;
}

// One table-build launch for every request admitted in a round: their
// descriptors are gathered device-to-device into one array, so the builds
// run side by side instead of one small launch after another.
qubo_status_t build_tables(qubo_server *s, const std::vector<Request *> &adm)
{
    if (adm.empty()) return QUBO_OK;
    int max_A = 0;
    for (size_t k = 0; k < adm.size(); k++) {
        QRT_HIP(hipMemcpyAsync(s->d_setup + k, adm[k]->job.d_insts, sizeof(qk::Inst),
                               hipMemcpyDeviceToDevice, s->stream),
                "hipMemcpyAsync descriptor");
        max_A = std::max(max_A, adm[k]->job.max_A);
    }
    QRT_HIP(qk::launch_tables(s->d_setup, int(adm.size()), max_A, nullptr, 0, s->stream),
            "tables kernel");
    return QUBO_OK;
}

// Enqueue one tick into buffer t; *launched stays false when there was nothing to do.
qubo_status_t enqueue_tick(qubo_server *s, TickBuf &t, bool *launched)
{
    *launched = false;
    std::vector<Request *> act;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        act = s->active;
    }
    // requests still owning unissued items or an unrun finish
    std::vector<Request *> walkers, finishers;
    for (Request *r : act) {
        const qplan::Plan &P = r->job.plans[0];
        if (P.direct) {
            if (r->next_item == 0) {   // not yet finished: finish-only request
                r->next_item = 1;
                finishers.push_back(r);
            }
        } else if (r->next_item < P.items) {
            walkers.push_back(r);
        }
    }
    // water-filling over the per-tick item budget, fewest remaining first,
    // then grouped by walk variant (one launch per variant group)
    std::sort(walkers.begin(), walkers.end(), [](Request *a, Request *b) {
        return a->job.plans[0].items - a->next_item < b->job.plans[0].items - b->next_item;
    });
    // Under a backlog the tick grows (qsched::tick_scale): fewer tick
    // boundaries (each costs a drain of the walk grid and a finish launch),
    // at no cost in latency since requests queue anyway.
    std::vector<uint64_t> left(walkers.size());
    for (size_t k = 0; k < walkers.size(); k++)
        left[k] = walkers[k]->job.plans[0].items - walkers[k]->next_item;
    const std::vector<uint64_t> share = qsched::tick_shares(left, s->tick_items);
    uint64_t total = 0;
    for (uint64_t c : share) total += c;
    if (total == 0 && finishers.empty()) return QUBO_OK;
    // descriptors grouped by variant; item numbering restarts in every group
    std::vector<size_t> idx(walkers.size());
    for (size_t k = 0; k < idx.size(); k++) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
        const qplan::Plan &a = walkers[x]->job.plans[0], &b = walkers[y]->job.plans[0];
        return std::make_tuple(a.mcols, a.vgpr_levels, a.tier) < std::make_tuple(b.mcols, b.vgpr_levels, b.tier);
    });
    struct Launch { int first, count; uint64_t items; const qplan::Plan *P; };
    std::vector<Launch> launches;
    int nw = 0;
    uint64_t g = 0;
    for (size_t k : idx) {
        Request *r = walkers[k];
        const uint64_t c = share[k];
        const qplan::Plan &P = r->job.plans[0];
        if (launches.empty() || !qrt::same_variant(*launches.back().P, P)) {
            launches.push_back({nw, 0, 0, &P});
            g = 0;
        }
        qk::Inst I = r->base;
        I.item_begin = g;
        I.item_end = g + c;
        I.item_local0 = r->next_item;
        I.res = r->base.res + r->next_item;
        I.bit0 = r->next_item;          // I.bits: the request's whole bitmap
        t.h_walk[nw++] = I;
        g += c;
        launches.back().count++;
        launches.back().items += c;
        r->next_item += c;
        if (r->next_item == P.items) finishers.push_back(r);
    }
    if (nw > 0) {
        QRT_HIP(hipMemcpyAsync(t.d_walk, t.h_walk, size_t(nw) * sizeof(qk::Inst), hipMemcpyHostToDevice,
                               s->stream),
                "hipMemcpyAsync tick");
        QRT_HIP(hipMemsetAsync(s->d_counter, 0, launches.size() * sizeof(unsigned long long), s->stream),
                "hipMemsetAsync");
        for (size_t k = 0; k < launches.size(); k++) {
            const Launch &L = launches[k];
            const int occ = qk::walk_occupancy(L.P->mcols, L.P->vgpr_levels, L.P->tier);
            const int waves = int(std::min<uint64_t>(L.items, uint64_t(s->cus) * uint64_t(occ)));
            QRT_HIP(qk::launch_walk(L.P->mcols, L.P->vgpr_levels, L.P->tier, t.d_walk + L.first, L.count,
                                    L.items, s->d_counter + k, s->d_karena, waves, s->stream),
                    "walk kernel");
        }
    }
    if (!finishers.empty()) {
        for (size_t i = 0; i < finishers.size(); i++) t.h_fin[i] = finishers[i]->base;
        QRT_HIP(hipMemcpyAsync(t.d_fin, t.h_fin, finishers.size() * sizeof(qk::Inst),
                               hipMemcpyHostToDevice, s->stream),
                "hipMemcpyAsync finish");
        QRT_HIP(qk::launch_finish(t.d_fin, int(finishers.size()), t.d_out, s->stream), "finish kernel");
        QRT_HIP(hipMemcpyAsync(t.h_out, t.d_out, finishers.size() * sizeof(qk::FinalRes),
                               hipMemcpyDeviceToHost, s->stream),
                "hipMemcpyAsync results");
    }
    t.finishing = std::move(finishers);
    QRT_HIP(hipEventRecord(t.done, s->stream), "hipEventRecord");
    t.inflight = true;
    *launched = true;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->n_ticks++;
    }
    return QUBO_OK;
}

void scheduler(qubo_server *s)
{
    if (hipSetDevice(s->dev) != hipSuccess) {
        fail_all(s, "hipSetDevice failed in the scheduler");
        return;
    }
    for (;;) {
        std::vector<Request *> adm;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            adm = take_admissions(s);
            const bool idle = adm.empty() && s->active.empty() && !s->ticks[0].inflight &&
                              !s->ticks[1].inflight;
            if (idle) {
                if (s->stop && s->queue.empty()) break;
                s->cv_work.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        for (Request *r : adm) {
            qubo_status_t st = setup_request(s, r);
            if (st != QUBO_OK) {
                fail_all(s, qrt::last_error_cstr());
                return;
            }
        }
        if (build_tables(s, adm) != QUBO_OK) {
            fail_all(s, qrt::last_error_cstr());
            return;
        }
        TickBuf &t = s->ticks[s->cur];
        if (t.inflight) {
            // the buffer's previous tick was enqueued two ticks ago
            if (hipEventSynchronize(t.done) != hipSuccess) {
                fail_all(s, "tick failed on the device");
                return;
            }
            complete_tick(s, t);
        }
        bool launched = false;
        if (enqueue_tick(s, t, &launched) != QUBO_OK) {
            fail_all(s, qrt::last_error_cstr());
            return;
        }
        if (launched) {
            s->cur ^= 1;
        } else {
            // nothing new to run: retire the other buffer's tick, if any
            TickBuf &o = s->ticks[s->cur ^ 1];
            if (o.inflight) {
                if (hipEventSynchronize(o.done) != hipSuccess) {
                    fail_all(s, "tick failed on the device");
                    return;
                }
                complete_tick(s, o);
            } else {
                std::unique_lock<std::mutex> lk(s->mu);
                if (s->queue.empty() || int(s->active.size()) >= s->max_slots)
                    s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
    }
}

void server_free(qubo_server *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (TickBuf &t : s->ticks) {
        if (t.done) (void)hipEventDestroy(t.done);
        if (t.h_walk) (void)hipHostFree(t.h_walk);
        if (t.h_fin) (void)hipHostFree(t.h_fin);
        if (t.h_out) (void)hipHostFree(t.h_out);
        if (t.d_walk) (void)hipFree(t.d_walk);
        if (t.d_fin) (void)hipFree(t.d_fin);
        if (t.d_out) (void)hipFree(t.d_out);
    }
    for (auto &kv : s->reqs) {
        if (kv.second->d_mem) (void)hipFree(kv.second->d_mem);
        delete kv.second;
    }
    if (s->d_karena) (void)hipFree(s->d_karena);
    if (s->d_setup) (void)hipFree(s->d_setup);
    if (s->d_counter) (void)hipFree(s->d_counter);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

qubo_status_t server_init(qubo_server *s, size_t budget, int max_slots)
{
    QRT_HIP(hipGetDevice(&s->dev), "hipGetDevice");
    s->budget = budget;
    s->max_slots = max_slots;
    qrt::DeviceInfo di;
    qubo_status_t st = qrt::device_info(&di);
    if (st != QUBO_OK) return st;
    s->cus = di.cus;
    // two items per resident wave of the default walk variant (B = 10, LDS
    // row cache): every wave of a tick then gets the same share, so the
    // tick ends without a half-idle tail
    s->tick_items = uint64_t(di.cus) * uint64_t(qk::walk_occupancy(16, 4, 2)) * 2;
    QRT_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
    QRT_HIP(hipMalloc(&s->d_karena, size_t(max_slots) * qk::kKTable * sizeof(int32_t)), "hipMalloc");
    QRT_HIP(hipMalloc(&s->d_setup, size_t(max_slots) * sizeof(qk::Inst)), "hipMalloc");
    // one item counter per walk variant launched in a tick
    QRT_HIP(hipMalloc(&s->d_counter, kMaxTickLaunches * sizeof(unsigned long long)), "hipMalloc");
    for (int k = max_slots - 1; k >= 0; k--) s->free_kslots.push_back(k);
    for (TickBuf &t : s->ticks) {
        QRT_HIP(hipEventCreateWithFlags(&t.done, hipEventDisableTiming), "hipEventCreate");
        const size_t ib = size_t(max_slots) * sizeof(qk::Inst), ob = size_t(max_slots) * sizeof(qk::FinalRes);
        QRT_HIP(hipHostMalloc(reinterpret_cast<void **>(&t.h_walk), ib, 0), "hipHostMalloc");
        QRT_HIP(hipHostMalloc(reinterpret_cast<void **>(&t.h_fin), ib, 0), "hipHostMalloc");
        QRT_HIP(hipHostMalloc(reinterpret_cast<void **>(&t.h_out), ob, 0), "hipHostMalloc");
        QRT_HIP(hipMalloc(&t.d_walk, ib), "hipMalloc");
        QRT_HIP(hipMalloc(&t.d_fin, ib), "hipMalloc");
        QRT_HIP(hipMalloc(&t.d_out, ob), "hipMalloc");
    }
    return QUBO_OK;
}

}  // namespace

extern "C" {

qubo_status_t qubo_server_create(size_t mem_budget_bytes, int max_slots, qubo_server_t **srv)
{
    try {
        qrt::set_error("");
        if (!srv || max_slots < 1 || max_slots > 65536 || mem_budget_bytes == 0) {
            qrt::set_error("bad server arguments");
            return QUBO_EINVAL;
        }
        qubo_server *s = new qubo_server();
        qubo_status_t st = server_init(s, mem_budget_bytes, max_slots);
        if (st != QUBO_OK) {
            const std::string keep = qrt::last_error_cstr();
            server_free(s);
            qrt::set_error(keep);
            return st;
        }
        s->th = std::thread(scheduler, s);
        *srv = s;
        return QUBO_OK;
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

qubo_status_t qubo_server_submit(qubo_server_t *s, const void *Q, int n, qubo_dtype_t dtype,
                                 uint64_t *ticket)
{
    try {
        qrt::set_error("");
        if (!s || !ticket) {
            qrt::set_error("null argument");
            return QUBO_EINVAL;
        }
        Request *r = new Request();
        r->job.plans.resize(1);
        std::string msg;
        qrt::tune_autoload();
        qubo_status_t st = qplan::make_plan(Q, n, dtype, nullptr, &r->job.plans[0], &msg, true);
        if (st != QUBO_OK) {
            delete r;
            qrt::set_error(msg);
            return st;
        }
        // Served requests walk 2^12-step items (a quarter of a batch's): a
        // tick then lasts about a millisecond at light load, which sets the
        // latency of a request that arrives while one runs; under a backlog
        // the ticks grow instead (enqueue_tick).  The planner's cap of 2^20
        // items per instance still holds (L >= A - 20), so large requests
        // keep their item records (16 B each) and their finish bounded.
        qplan::Plan &P = r->job.plans[0];
        const int serveL = std::max(kServeL, P.A - 20);
        if (!P.direct && P.L > serveL) {
            P.L = serveL;
            P.items = uint64_t(1) << (P.A - P.L);
        }
        if (dtype == QUBO_FP32) {
            const float *q = static_cast<const float *>(Q);
            r->qf.assign(q, q + size_t(n) * n);
            r->job.qf.push_back(r->qf.data());
        } else {
            r->job.qf.push_back(nullptr);
        }
        st = qrt::job_layout(&r->job, 0);
        if (st != QUBO_OK) {
            delete r;
            return st;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->fatal.empty()) {
            delete r;
            qrt::set_error(s->fatal);
            return QUBO_EDEVICE;
        }
        if (r->job.bytes > s->budget) {
            delete r;
            qrt::set_error("request needs more device memory than the server budget");
            return QUBO_ENOMEM;
        }
        r->ticket = s->next_ticket++;
        r->arrival = Clock::now();
        if (!s->have_t0) {
            s->have_t0 = true;
            s->t0 = r->arrival;
        }
        s->reqs[r->ticket] = r;
        s->queue.push_back(r);
        *ticket = r->ticket;
        s->cv_work.notify_one();
        return QUBO_OK;
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

static qubo_status_t take_result(qubo_server *s, uint64_t ticket, qubo_result_t *out, bool *ready)
{
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        qrt::set_error("unknown ticket");
        *ready = true;
        return QUBO_EINVAL;
    }
    Request *r = it->second;
    if (r->state == RState::Queued || r->state == RState::Active) {
        *ready = false;
        return QUBO_EAGAIN;
    }
    *ready = true;
    qubo_status_t st = r->status;
    if (r->state == RState::Done) {
        if (out) *out = r->result;
    } else {
        qrt::set_error(r->error);
    }
    s->reqs.erase(it);
    delete r;
    return st;
}

qubo_status_t qubo_server_poll(qubo_server_t *s, uint64_t ticket, qubo_result_t *out)
{
    if (!s) {
        qrt::set_error("null server");
        return QUBO_EINVAL;
    }
    qrt::set_error("");
    std::lock_guard<std::mutex> lk(s->mu);
    bool ready = false;
    return take_result(s, ticket, out, &ready);
}

qubo_status_t qubo_server_wait(qubo_server_t *s, uint64_t ticket, double timeout_ms,
                               qubo_result_t *out)
{
    if (!s) {
        qrt::set_error("null server");
        return QUBO_EINVAL;
    }
    qrt::set_error("");
    const auto deadline = Clock::now() + std::chrono::microseconds(int64_t(timeout_ms * 1000.0));
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool ready = false;
        qubo_status_t st = take_result(s, ticket, out, &ready);
        if (ready) return st;
        if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            st = take_result(s, ticket, out, &ready);
            return st;
        }
    }
}

qubo_status_t qubo_server_stats(qubo_server_t *s, double *p50_ms, double *p99_ms,
                                double *states_per_s)
{
    if (!s) {
        qrt::set_error("null server");
        return QUBO_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
        if (v.empty()) return 0.0;
        // nearest-rank percentile
        size_t k = size_t(std::ceil(p / 100.0 * double(v.size())));
        if (k < 1) k = 1;
        return v[k - 1];
    };
    if (p50_ms) *p50_ms = pct(50.0);
    if (p99_ms) *p99_ms = pct(99.0);
    if (states_per_s) {
        const double sec = s->have_t0 ? ms_since(s->t0) / 1e3 : 0.0;
        *states_per_s = sec > 0 ? s->states_done / sec : 0.0;
    }
    return QUBO_OK;
}

qubo_status_t qubo_server_info(qubo_server_t *s, size_t *mem_in_use, size_t *mem_peak,
                               int *active_peak, uint64_t *ticks)
{
    if (!s) {
        qrt::set_error("null server");
        return QUBO_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (mem_in_use) *mem_in_use = s->mem_used;
    if (mem_peak) *mem_peak = s->mem_peak;
    if (active_peak) *active_peak = s->active_peak;
    if (ticks) *ticks = s->n_ticks;
    return QUBO_OK;
}

void qubo_server_destroy(qubo_server_t *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    server_free(s);
}

}  // extern "C"

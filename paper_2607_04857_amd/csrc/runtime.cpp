// runtime.cpp -- device jobs and the single-instance C ABI.
#include "runtime.h"

#include <chrono>
#include <cmath>
#include <cstring>
#include <algorithm>
#include <mutex>

static_assert(qk::kMaxVars == qplan::kMaxN, "finish kernel LDS sized for the largest n");
static_assert(qk::kExactSumLimit == qplan::kIntSumLimit, "one int32 exactness bound");
static_assert(qk::kPackSumLimit == qplan::kPackSumLimit, "one packed-tier bound");

namespace qrt {

namespace {
thread_local std::string g_last_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct JobOffsets {
    size_t insts = 0, counter = 0, res = 0, out = 0, K = 0, gbest = 0, prep = 0;
    std::vector<size_t> T, Qf, M, EB, S, bits;
    // top-k (k > 1, one instance)
    size_t gthr = 0, hist = 0, lowbin = 0, candN = 0, candE = 0, candR = 0, listE = 0, listR = 0, listCount = 0, chunkE = 0, chunkR = 0, chunkCount = 0,
           stE = 0, stI = 0, segCount = 0, selE = 0, selR = 0, selCount = 0, topk = 0;
};

}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

const char *last_error_cstr() { return g_last_error.c_str(); }

qubo_status_t device_error(const char *what, hipError_t e)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return QUBO_EDEVICE;
}

qubo_status_t device_info(DeviceInfo *info)
{
    int dev = 0;
    QRT_HIP(hipGetDevice(&dev), "hipGetDevice");
    static std::mutex mu;
    static int cached_dev = -1, cached_cus = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (cached_dev != dev) {
            hipDeviceProp_t prop;
            QRT_HIP(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
            cached_dev = dev;
            cached_cus = prop.multiProcessorCount;
        }
        info->device = dev;
        info->cus = cached_cus;
    }
    return QUBO_OK;
}

}  // namespace qrt

// Layout helpers kept in one translation unit with the job code.
namespace qrt {

static JobOffsets compute_offsets(const Job &job, size_t *stage_bytes, size_t *bytes)
{
    JobOffsets o;
    const size_t ni = job.plans.size();
    size_t off = 0;
    o.insts = off;
    off = align_up(off + ni * sizeof(qk::Inst), 256);
    for (size_t i = 0; i < ni; i++) {
        const size_t nn = size_t(job.plans[i].n) * job.plans[i].n;
        o.T.push_back(off);
        off = align_up(off + nn * sizeof(int32_t), 256);
        if (job.qf[i]) {
            o.Qf.push_back(off);
            off = align_up(off + nn * sizeof(float), 256);
        } else {
            o.Qf.push_back(size_t(-1));
        }
    }
    const size_t k = size_t(job.topk);
    if (k > 1) {   // the shared top-k bound and histogram start in the uploaded image
        o.gthr = off;
        off = align_up(off + sizeof(int32_t), 256);
        o.lowbin = off;
        off = align_up(off + sizeof(int32_t), 256);
        o.candN = off;
        off = align_up(off + sizeof(int32_t), 256);
        o.hist = off;
        off = align_up(off + qk::kTopkBins * sizeof(uint32_t), 256);
    }
    *stage_bytes = off;
    o.counter = off;
    off = align_up(off + std::max<size_t>(1, job.groups.size()) * sizeof(unsigned long long), 256);
    for (size_t i = 0; i < ni; i++) {
        const qplan::Plan &P = job.plans[i];
        // words per M_int row: 2^B, or 2^(B-1) packed (two columns a word)
        const size_t A = P.direct ? 0 : size_t(P.A),
                     NS = P.direct ? 0 : (size_t(1) << (P.tier >= 4 ? P.B - 1 : P.B));
        // M_int and the prefix couplings, each followed by its negation
        o.M.push_back(off);
        off = align_up(off + 2 * A * NS * sizeof(int32_t), 256);
        o.EB.push_back(off);
        off = align_up(off + NS * sizeof(int32_t), 256);
        o.S.push_back(off);
        off = align_up(off + 2 * A * qk::kWave * sizeof(int32_t), 256);
    }
    o.K = off;
    off = align_up(off + ni * qk::kKTable * sizeof(int32_t), 256);
    o.res = off;
    off = align_up(off + size_t(job.total_items) * sizeof(qk::ItemRes), 256);
    // one bit per item record of each instance (which records were written)
    for (size_t i = 0; i < ni; i++) {
        const qplan::Plan &P = job.plans[i];
        const size_t words = P.direct ? 0 : size_t((P.walk_items() + 31) / 32);
        o.bits.push_back(off);
        off = align_up(off + std::max<size_t>(words, 1) * sizeof(uint32_t), 256);
    }
    o.out = off;
    off = align_up(off + ni * sizeof(qk::FinalRes), 256);
    o.gbest = off;
    off = align_up(off + ni * sizeof(int32_t), 256);
    o.prep = off;
    off = align_up(off + sizeof(qk::PrepOut), 256);
    if (k > 1) {
        const qplan::Plan &P = job.plans[0];
        const size_t W = job.groups.empty() ? 0 : size_t(job.groups[0].waves);
        const size_t nst = P.direct ? (size_t(1) << P.n) : (k << P.B);
        auto put = [&](size_t *field, size_t bytes_) {
            *field = off;
            off = align_up(off + std::max<size_t>(bytes_, 1), 256);
        };
        put(&o.listE, W * k * sizeof(int32_t));
        put(&o.listR, W * k * sizeof(uint64_t));
        put(&o.listCount, W * sizeof(int32_t));
        put(&o.candE, W * k * sizeof(int32_t));
        put(&o.candR, W * k * sizeof(uint64_t));
        put(&o.chunkE, k * sizeof(int32_t));
        put(&o.chunkR, k * sizeof(uint64_t));
        put(&o.chunkCount, sizeof(int32_t));
        put(&o.stE, nst * sizeof(int32_t));
        put(&o.stI, nst * sizeof(uint64_t));
        put(&o.segCount, k * sizeof(int32_t));
        put(&o.selE, k * sizeof(int32_t));
        put(&o.selR, k * sizeof(uint64_t));
        put(&o.selCount, sizeof(int32_t));
        put(&o.topk, k * sizeof(qk::TopkState));
    }
    *bytes = off;
    return o;
}

bool same_variant(const qplan::Plan &a, const qplan::Plan &b)
{
    return a.mcols == b.mcols && a.vgpr_levels == b.vgpr_levels && a.tier == b.tier;
}

qubo_status_t job_layout(Job *job, int waves_per_cu)
{
    job->max_A = 0;
    job->total_items = 0;
    job->states = 0.0;
    job->groups.clear();
    DeviceInfo di;
    qubo_status_t st = device_info(&di);
    if (st != QUBO_OK) return st;
    for (size_t i = 0; i < job->plans.size(); i++) {
        const qplan::Plan &P = job->plans[i];
        job->states += std::ldexp(1.0, P.n);
        if (P.direct) continue;
        if (job->groups.empty() || !same_variant(job->plans[size_t(job->groups.back().first)], P) ||
            size_t(job->groups.back().first + job->groups.back().count) != i) {
            if (!qk::walk_variant_exists(P.mcols, P.vgpr_levels)) {
                set_error("no walk kernel built for this B / vgpr_levels");
                return QUBO_EINVAL;
            }
            WalkGroup g;
            g.first = int(i);
            g.mcols = P.mcols;
            g.vgpr_levels = P.vgpr_levels;
            g.tier = P.tier;
            job->groups.push_back(g);
        }
        WalkGroup &g = job->groups.back();
        g.count = int(i) + 1 - g.first;
        g.items += P.walk_items();
        if (P.A > job->max_A) job->max_A = P.A;
        job->total_items += P.walk_items();
    }
    if (job->topk > 1 && (job->plans.size() != 1 ||
                          (!job->groups.empty() && job->groups[0].tier != 3 && job->groups[0].tier != 5))) {
        set_error("internal: top-k jobs hold one instance planned for tier 3 or 5");
        return QUBO_EINTERNAL;
    }
    for (WalkGroup &g : job->groups) {
        int wpc = waves_per_cu > 0 ? waves_per_cu
                                   : qk::walk_occupancy(g.mcols, g.vgpr_levels, g.tier, job->topk);
        if (wpc <= 0) wpc = 1;
        uint64_t waves = uint64_t(di.cus) * uint64_t(wpc);
        if (g.items < waves) waves = g.items;
        g.waves = int(waves);
    }
    size_t sb = 0, b = 0;
    (void)compute_offsets(*job, &sb, &b);
    job->stage_bytes = sb;
    job->bytes = b;
    return QUBO_OK;
}

// Fill the staging image and device pointers for allocation d_mem.
qubo_status_t job_bind(Job *job, void *d_mem)
{
    size_t sb = 0, b = 0;
    JobOffsets o = compute_offsets(*job, &sb, &b);
    unsigned char *base = static_cast<unsigned char *>(d_mem);
    job->d_mem = d_mem;
    job->stage.assign(sb, 0);
    job->d_insts = reinterpret_cast<qk::Inst *>(base + o.insts);
    job->d_counter = reinterpret_cast<unsigned long long *>(base + o.counter);
    job->d_res = reinterpret_cast<qk::ItemRes *>(base + o.res);
    job->d_out = reinterpret_cast<qk::FinalRes *>(base + o.out);
    job->d_k = reinterpret_cast<int32_t *>(base + o.K);
    job->d_prep = job->dq ? reinterpret_cast<qk::PrepOut *>(base + o.prep) : nullptr;
    job->d_T0 = reinterpret_cast<int32_t *>(base + o.T[0]);
    std::vector<qk::Inst> insts(job->plans.size());
    uint64_t item = 0;        // result slot of the instance's first item (whole job)
    // walk numbering restarts at 0 in every group
    std::vector<uint64_t> group_base(job->plans.size(), 0);
    for (const WalkGroup &g : job->groups) {
        uint64_t acc = 0;
        for (int k = g.first; k < g.first + g.count; k++) {
            group_base[size_t(k)] = acc;
            acc += job->plans[size_t(k)].walk_items();
        }
    }
    for (size_t i = 0; i < job->plans.size(); i++) {
        const qplan::Plan &P = job->plans[i];
        qk::Inst &I = insts[i];
        I.T = reinterpret_cast<const int32_t *>(base + o.T[i]);
        I.M = reinterpret_cast<int32_t *>(base + o.M[i]);
        I.EB = reinterpret_cast<int32_t *>(base + o.EB[i]);
        I.S = reinterpret_cast<int32_t *>(base + o.S[i]);
        I.K = reinterpret_cast<int32_t *>(base + o.K) + i * qk::kKTable;
        I.Qf = job->qf[i] ? reinterpret_cast<const float *>(base + o.Qf[i]) : nullptr;
        I.res = job->d_res + item;
        I.bits = P.direct ? nullptr : reinterpret_cast<uint32_t *>(base + o.bits[i]);
        I.bit0 = 0;
        I.n = P.n;
        I.A = P.A;
        I.B = P.B;
        I.L = P.L;
        I.direct = P.direct ? 1 : 0;
        I.kslot = int(i);
        I.packed = (P.tier == 4 || P.tier == 5) ? 1 : 0;
        I.pack_shift = P.direct ? 0 : P.pack_shift;   // device-prepared: set by prepare_kernel
        I.item_begin = group_base[i];
        I.item_end = group_base[i] + (P.direct ? 0 : P.walk_items());
        item += P.direct ? 0 : P.walk_items();
        I.item_local0 = P.item_first;
        I.n_items = P.direct ? 0 : P.walk_items();
        I.gbest = reinterpret_cast<int32_t *>(base + o.gbest) + i;
        I.prep = job->d_prep;
        const size_t nn = size_t(P.n) * P.n;
        if (job->dq) {
            // T is written by the prepare kernel; the float64 rescore reads
            // the caller's matrix where it is
            if (P.dtype == QUBO_FP32) I.Qf = static_cast<const float *>(job->dq);
        } else {
            std::memcpy(job->stage.data() + o.T[i], P.T.data(), nn * sizeof(int32_t));
        }
        if (job->qf[i]) std::memcpy(job->stage.data() + o.Qf[i], job->qf[i], nn * sizeof(float));
    }
    std::memcpy(job->stage.data() + o.insts, insts.data(), insts.size() * sizeof(qk::Inst));
    if (job->topk > 1) {
        const int32_t none = qk::kNoEnergy, nobin = qk::kTopkBins;
        std::memcpy(job->stage.data() + o.gthr, &none, sizeof(none));
        std::memcpy(job->stage.data() + o.lowbin, &nobin, sizeof(nobin));
        qk::TopkBufs &t = job->tkb;
        t.walk.listE = reinterpret_cast<int32_t *>(base + o.listE);
        t.walk.listR = reinterpret_cast<uint64_t *>(base + o.listR);
        t.walk.listCount = reinterpret_cast<int32_t *>(base + o.listCount);
        t.walk.gthr = reinterpret_cast<int32_t *>(base + o.gthr);
        t.walk.hist = reinterpret_cast<uint32_t *>(base + o.hist);
        t.walk.lowbin = reinterpret_cast<int32_t *>(base + o.lowbin);
        // bins of (E + sum|T|) over [0, 2 sum|T|]
        const int64_t span = 2 * job->plans[0].sum_abs;
        int shift = 0;
        while ((span >> shift) >= qk::kTopkBins) shift++;
        t.walk.hist_lo = -job->plans[0].sum_abs;
        t.walk.hist_shift = shift;
        t.walk.prep = job->d_prep;   // device-prepared: the bins from the preparation
        t.walk.k = job->topk;
        t.waves = job->groups.empty() ? 0 : job->groups[0].waves;
        t.candE = reinterpret_cast<int32_t *>(base + o.candE);
        t.candR = reinterpret_cast<uint64_t *>(base + o.candR);
        t.candN = reinterpret_cast<int32_t *>(base + o.candN);
        t.chunkE = reinterpret_cast<int32_t *>(base + o.chunkE);
        t.chunkR = reinterpret_cast<uint64_t *>(base + o.chunkR);
        t.chunkCount = reinterpret_cast<int32_t *>(base + o.chunkCount);
        t.stE = reinterpret_cast<int32_t *>(base + o.stE);
        t.stI = reinterpret_cast<uint64_t *>(base + o.stI);
        t.segCount = reinterpret_cast<int32_t *>(base + o.segCount);
        t.selE = reinterpret_cast<int32_t *>(base + o.selE);
        t.selR = reinterpret_cast<uint64_t *>(base + o.selR);
        t.selCount = reinterpret_cast<int32_t *>(base + o.selCount);
        t.out = reinterpret_cast<qk::TopkState *>(base + o.topk);
        job->h_inst0 = insts[0];
    }
    return QUBO_OK;
}

qubo_status_t job_enqueue_kernels(const Job &job, hipStream_t stream, hipEvent_t walk_begin,
                                  hipEvent_t walk_end)
{
    const int ni = int(job.plans.size());
    if (job.dq)
        QRT_HIP(qk::launch_prepare(job.dq, job.plans[0].n, job.plans[0].dtype == QUBO_FP32 ? 1 : 0,
                                   job.d_T0, job.d_prep, job.d_insts, stream),
                "prepare kernel");
    QRT_HIP(qk::launch_tables(job.d_insts, ni, job.max_A, job.d_counter, int(job.groups.size()),
                              stream),
            "tables kernel");
    if (walk_begin) QRT_HIP(hipEventRecord(walk_begin, stream), "hipEventRecord");
    if (job.topk > 1) {
        // a bound of the k-th smallest chunk key from states near a local
        // minimum, when the walk covers every chunk (timed with the walk)
        const qk::Inst &I = job.h_inst0;
        if (!I.direct && I.item_local0 == 0 && I.n_items == (uint64_t(1) << (I.A - I.L)))
            QRT_HIP(qk::launch_topk_seed(job.d_insts, job.tkb.walk.gthr, job.topk, stream),
                    "top-k seed kernel");
    }
    for (size_t k = 0; k < job.groups.size(); k++) {
        const WalkGroup &g = job.groups[k];
        QRT_HIP(qk::launch_walk(g.mcols, g.vgpr_levels, g.tier, job.d_insts + g.first, g.count,
                                g.items, job.d_counter + k, job.d_k, g.waves, stream,
                                job.topk > 1 ? &job.tkb.walk : nullptr),
                "walk kernel");
    }
    if (walk_end) QRT_HIP(hipEventRecord(walk_end, stream), "hipEventRecord");
    if (job.topk > 1)
        QRT_HIP(qk::launch_topk_finish(job.d_insts, job.h_inst0, job.tkb, job.topk, job.d_out, stream),
                "top-k kernels");
    else
        QRT_HIP(qk::launch_finish(job.d_insts, ni, job.d_out, stream), "finish kernel");
    return QUBO_OK;
}

qubo_status_t job_result(const Job &job, int i, const qk::FinalRes &fr, qubo_result_t *out)
{
    const qplan::Plan &P = job.plans[size_t(i)];
    if (fr.status != 0) {
        set_error("internal self-check failed (status " + std::to_string(fr.status) + ")");
        return QUBO_EINTERNAL;
    }
    std::memset(out, 0, sizeof(*out));
    out->best.energy_i = fr.E;
    out->best.index = fr.index;
    out->best.energy = (P.dtype == QUBO_FP32) ? fr.E64 : double(fr.E);
    out->tol = (P.dtype == QUBO_FP32) ? 2.0 * P.eps_q : 0.0;
    out->p = P.p;
    out->A = P.direct ? P.n : P.A;
    out->B = P.B;
    out->L = P.L;
    out->tier = P.tier;
    out->vgpr_levels = P.direct ? 0 : P.vgpr_levels;
    out->states = (P.n >= 64) ? ~0ull : (1ull << P.n);
    return QUBO_OK;
}

}  // namespace qrt

// ------------------------------------------------------------------ C ABI

namespace qrt {

hipStream_t thread_stream(qubo_status_t *st)
{
    thread_local hipStream_t s = nullptr;
    thread_local int dev = -1;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) {
        *st = qrt::device_error("hipGetDevice", hipErrorNoDevice);
        return nullptr;
    }
    if (!s || dev != cur) {
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            *st = qrt::device_error("hipStreamCreate", e);
            s = nullptr;
            return nullptr;
        }
        dev = cur;
    }
    *st = QUBO_OK;
    return s;
}

qubo_status_t solve_planned(qrt::Job &job, hipStream_t stream, int waves_per_cu, qubo_result_t *out,
                            qubo_state_t *topk)
{
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    qubo_status_t st = qrt::job_layout(&job, waves_per_cu);
    if (st != QUBO_OK) return st;
    void *d_mem = nullptr;
    QRT_HIP(hipMallocAsync(&d_mem, job.bytes, stream), "hipMallocAsync");
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    qubo_status_t rs = QUBO_OK;
    qk::FinalRes fr{};
    qk::PrepOut prep{};
    std::vector<qk::TopkState> tk_host;
    do {
        if ((rs = qrt::job_bind(&job, d_mem)) != QUBO_OK) break;
        hipError_t e;
        if ((e = hipEventCreate(&ev0)) != hipSuccess || (e = hipEventCreate(&ev1)) != hipSuccess) {
            rs = qrt::device_error("hipEventCreate", e);
            break;
        }
        if ((e = hipMemcpyAsync(d_mem, job.stage.data(), job.stage_bytes, hipMemcpyHostToDevice,
                                stream)) != hipSuccess) {
            rs = qrt::device_error("hipMemcpyAsync H2D", e);
            break;
        }
        if ((rs = qrt::job_enqueue_kernels(job, stream, ev0, ev1)) != QUBO_OK) break;
        if ((e = hipMemcpyAsync(&fr, job.d_out, sizeof(fr), hipMemcpyDeviceToHost, stream)) !=
            hipSuccess) {
            rs = qrt::device_error("hipMemcpyAsync D2H", e);
            break;
        }
        if (job.dq && (e = hipMemcpyAsync(&prep, job.d_prep, sizeof(prep), hipMemcpyDeviceToHost,
                                          stream)) != hipSuccess) {
            rs = qrt::device_error("hipMemcpyAsync D2H preparation", e);
            break;
        }
        if (job.topk > 1) {
            static_assert(sizeof(qk::TopkState) == sizeof(qubo_state_t), "top-k state layout");
            tk_host.resize(size_t(job.topk));
            if ((e = hipMemcpyAsync(tk_host.data(), job.tkb.out, tk_host.size() * sizeof(qk::TopkState),
                                    hipMemcpyDeviceToHost, stream)) != hipSuccess) {
                rs = qrt::device_error("hipMemcpyAsync D2H top-k", e);
                break;
            }
        }
    } while (false);
    hipError_t ef = hipFreeAsync(d_mem, stream);
    hipError_t es = hipStreamSynchronize(stream);
    float ms = 0.f;
    if (rs == QUBO_OK && es == hipSuccess) (void)hipEventElapsedTime(&ms, ev0, ev1);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (rs != QUBO_OK) return rs;
    if (es != hipSuccess) return qrt::device_error("hipStreamSynchronize", es);
    if (ef != hipSuccess) return qrt::device_error("hipFreeAsync", ef);
    if (job.dq) {
        // the device preparation's outcome for the input, as the host planner's
        switch (prep.status) {
        case 0: break;
        case qk::kPrepOverflow:
            qrt::set_error("sum of |T_ij| exceeds 2^30 - 1: int32 walk not provably exact");
            return QUBO_EOVERFLOW;
        case qk::kPrepNonFinite:
            qrt::set_error("non-finite entry in Q");
            return QUBO_ENONFINITE;
        default:
            qrt::set_error("internal: scaled matrix exceeds the int32 bound");
            return QUBO_EINTERNAL;
        }
        qplan::Plan &P = job.plans[0];
        P.p = prep.p;
        P.eps_q = prep.eps_q;
        P.sum_abs = prep.sum_abs;
    }
    st = qrt::job_result(job, 0, fr, out);
    if (st != QUBO_OK) return st;
    if (job.topk > 1 && topk) {
        const bool fp = job.plans[0].dtype == QUBO_FP32;
        for (int i = 0; i < job.topk; i++) {
            topk[i].energy_i = tk_host[size_t(i)].E;
            topk[i].index = tk_host[size_t(i)].index;
            topk[i].energy = fp ? tk_host[size_t(i)].E64 : double(tk_host[size_t(i)].E);
        }
    }
    out->kernel_ms = ms;
    out->total_ms = std::chrono::duration<double, std::milli>(clock::now() - t0).count();
    return QUBO_OK;
}

}  // namespace qrt

namespace {

using qrt::solve_planned;
using qrt::thread_stream;

qubo_status_t check_k(int k, int n, qubo_state_t *topk)
{
    if (k < 0 || k > 1024) {
        qrt::set_error("k must be in [0, 1024]");
        return QUBO_EINVAL;
    }
    if (k > 1) {
        if (!topk) {
            qrt::set_error("topk output required for k > 1");
            return QUBO_EINVAL;
        }
        if (n >= 1 && n < 11 && (1 << n) < k) {
            qrt::set_error("k exceeds the number of states");
            return QUBO_EINVAL;
        }
    }
    return QUBO_OK;
}

// The top-k walk keeps candidate lists (tier 3, or 5 on the packed layout);
// the finish selects.
void plan_topk(qrt::Job &job, int k, const qubo_options_t *opt)
{
    job.topk = k;
    qplan::Plan &P = job.plans[0];
    if (P.direct) return;
    P.tier = P.tier == 4 ? 5 : 3;
    const int t = P.tier;
    // The list entries live in global memory and only their scalars in LDS,
    // so the LDS row caches keep four waves per SIMD for any k.  With the
    // seeded bound the default one ("4") is the fastest top-k walk (its one
    // spilled register is reloaded once per super-block); "3" is next, and
    // the VGPR row cache (three waves) is taken should neither fit four waves.
    if ((P.vgpr_levels == 4 || P.vgpr_levels == 3) && !(opt && opt->vgpr_levels)) {
        if (qk::walk_occupancy(P.mcols, 4, t, k) >= 4 * 4) P.vgpr_levels = 4;
        else P.vgpr_levels = qk::walk_occupancy(P.mcols, 3, t, k) >= 4 * 4 ? 3 : 6;
    }
}

qubo_status_t solve_host(const void *Q, int n, qubo_dtype_t dtype, int k, const qubo_options_t *opt,
                         hipStream_t stream, qubo_result_t *out, qubo_state_t *topk)
{
    if (!out) {
        qrt::set_error("null output");
        return QUBO_EINVAL;
    }
    qubo_status_t st = check_k(k, n, topk);
    if (st != QUBO_OK) return st;
    qrt::tune_autoload();
    qrt::Job job;
    job.plans.resize(1);
    std::string msg;
    st = qplan::make_plan(Q, n, dtype, opt, &job.plans[0], &msg);
    if (st != QUBO_OK) {
        qrt::set_error(msg);
        return st;
    }
    job.qf.push_back(dtype == QUBO_FP32 ? static_cast<const float *>(Q) : nullptr);
    if (k > 1) plan_topk(job, k, opt);
    st = solve_planned(job, stream, opt ? opt->waves_per_cu : 0, out, topk);
    if (st == QUBO_OK && k == 1 && topk) topk[0] = out->best;
    return st;
}

}  // namespace

extern "C" {

qubo_status_t qubo_solve_ex(const void *Q, int n, qubo_dtype_t dtype, int k,
                            const qubo_options_t *opt, qubo_result_t *out, qubo_state_t *topk)
{
    try {
        qrt::set_error("");
        qubo_status_t st = check_k(k, n, topk);
        if (st != QUBO_OK) return st;
        hipStream_t s = thread_stream(&st);
        if (st != QUBO_OK) return st;
        return solve_host(Q, n, dtype, k, opt, s, out, topk);
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

qubo_status_t qubo_solve(const void *Q, int n, qubo_dtype_t dtype, int k, qubo_result_t *out,
                         qubo_state_t *topk)
{
    return qubo_solve_ex(Q, n, dtype, k, nullptr, out, topk);
}

qubo_status_t qubo_solve_device(const void *dQ, int n, qubo_dtype_t dtype, int k, void *hip_stream,
                                qubo_result_t *out, qubo_state_t *topk)
{
    try {
        qrt::set_error("");
        if (!dQ || n < 1 || n > qplan::kMaxN) {
            qrt::set_error("bad device Q or n");
            return QUBO_EINVAL;
        }
        qubo_status_t st = check_k(k, n, topk);
        if (st != QUBO_OK) return st;
        if (!out) {
            qrt::set_error("null output");
            return QUBO_EINVAL;
        }
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        // The plan depends on n, dtype and the tuning table only; the fold,
        // the exactness proof and the float32 scaling run on the device, in
        // stream order after whatever wrote dQ, and their outcome comes back
        // with the answer (one synchronisation, at the end).
        qrt::tune_autoload();
        qrt::Job job;
        job.plans.resize(1);
        std::string msg;
        st = qplan::make_plan_shape(n, dtype, nullptr, &job.plans[0], &msg);
        if (st != QUBO_OK) {
            qrt::set_error(msg);
            return st;
        }
        job.qf.push_back(nullptr);
        job.dq = dQ;
        if (k > 1) plan_topk(job, k, nullptr);
        st = solve_planned(job, s, 0, out, topk);
        if (st == QUBO_OK && k == 1 && topk) topk[0] = out->best;
        return st;
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

qubo_status_t qubo_plan_info(const void *Q, int n, qubo_dtype_t dtype, const qubo_options_t *opt,
                             qubo_plan_info_t *info, int32_t *T_out)
{
    try {
        qrt::set_error("");
        if (!info) {
            qrt::set_error("null info");
            return QUBO_EINVAL;
        }
        qplan::Plan P;
        std::string msg;
        qubo_status_t st = qplan::make_plan(Q, n, dtype, opt, &P, &msg);
        if (st != QUBO_OK) {
            qrt::set_error(msg);
            return st;
        }
        info->n = P.n;
        info->A = P.A;
        info->B = P.B;
        info->L = P.L;
        info->tier = P.tier;
        info->direct = P.direct ? 1 : 0;
        info->vgpr_levels = P.vgpr_levels;
        info->p = P.p;
        info->eps_q = P.eps_q;
        info->sum_abs_t = P.sum_abs;
        info->items = P.items;
        info->pack_shift = P.direct ? 0 : P.pack_shift;
        info->reserved = 0;
        if (T_out) std::memcpy(T_out, P.T.data(), P.T.size() * sizeof(int32_t));
        return QUBO_OK;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

const char *qubo_last_error(void) { return qrt::last_error_cstr(); }

const char *qubo_version(void) { return "qubo-mi355x 0.1"; }

}  // extern "C"

// batch.cpp -- many independent instances in one persistent walk launch.
//
// Every instance is planned on the host, laid out in one device allocation,
// and its work items are queued largest instance first (longest-processing-
// time order), so the persistent walk grid drains the big instances while
// the small ones fill the tail.  The H2D upload, table build, walk, per-
// instance finish and D2H download are captured once into a HIP graph and
// replayed by qubo_batch_run.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <tuple>

#include "runtime.h"

struct qubo_batch {
    qrt::Job job;
    std::vector<int> order;                    // walk position -> caller's index
    std::vector<std::vector<float>> qf_copy;   // owned float32 inputs
    hipStream_t stream = nullptr;
    void *d_mem = nullptr;
    unsigned char *h_stage = nullptr;          // pinned staging image
    qk::FinalRes *h_out = nullptr;             // pinned results
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float last_ms = 0.f;
    bool ran = false;
};

namespace {

void batch_free(qubo_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->d_mem) (void)hipFree(b->d_mem);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->h_out) (void)hipHostFree(b->h_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

qubo_status_t batch_build(qubo_batch *b, int count, const void *const *Q, const int *n,
                          const qubo_dtype_t *dtype, const qubo_options_t *opt)
{
    if (opt && (opt->item_first || opt->item_count)) {
        qrt::set_error("item ranges are for single solves");
        return QUBO_EINVAL;
    }
    std::vector<qplan::Plan> plans(static_cast<size_t>(count));
    std::string msg;
    qrt::tune_autoload();
    for (int i = 0; i < count; i++) {
        if (!Q[i]) {
            qrt::set_error("null Q in batch at " + std::to_string(i));
            return QUBO_EINVAL;
        }
        qubo_status_t st = qplan::make_plan(Q[i], n[i], dtype[i], opt, &plans[size_t(i)], &msg, true);
        if (st != QUBO_OK) {
            qrt::set_error("instance " + std::to_string(i) + ": " + msg);
            return st;
        }
    }
    // Walk order: grouped by walk kernel variant (one persistent launch per
    // group), most walk work first inside a group; direct (tiny) instances last.
    b->order.resize(size_t(count));
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        const qplan::Plan &px = plans[size_t(x)], &py = plans[size_t(y)];
        if (px.direct != py.direct) return !px.direct;
        const auto kx = std::make_tuple(px.mcols, px.vgpr_levels, px.tier);
        const auto ky = std::make_tuple(py.mcols, py.vgpr_levels, py.tier);
        if (kx != ky) return kx > ky;
        return px.n > py.n;
    });
    b->qf_copy.resize(size_t(count));
    for (int w = 0; w < count; w++) {
        const int i = b->order[size_t(w)];
        b->job.plans.push_back(std::move(plans[size_t(i)]));
        if (dtype[i] == QUBO_FP32) {
            const float *q = static_cast<const float *>(Q[i]);
            b->qf_copy[size_t(w)].assign(q, q + size_t(n[i]) * n[i]);
            b->job.qf.push_back(b->qf_copy[size_t(w)].data());
        } else {
            b->job.qf.push_back(nullptr);
        }
    }
    qubo_status_t st = qrt::job_layout(&b->job, opt ? opt->waves_per_cu : 0);
    if (st != QUBO_OK) return st;
    QRT_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "hipStreamCreate");
    QRT_HIP(hipEventCreate(&b->ev0), "hipEventCreate");
    QRT_HIP(hipEventCreate(&b->ev1), "hipEventCreate");
    hipError_t e = hipMalloc(&b->d_mem, b->job.bytes);
    if (e != hipSuccess) {
        b->d_mem = nullptr;
        qrt::set_error("device allocation of " + std::to_string(b->job.bytes) + " bytes failed");
        return QUBO_ENOMEM;
    }
    st = qrt::job_bind(&b->job, b->d_mem);
    if (st != QUBO_OK) return st;
    QRT_HIP(hipHostMalloc(reinterpret_cast<void **>(&b->h_stage), b->job.stage_bytes, 0),
            "hipHostMalloc");
    std::memcpy(b->h_stage, b->job.stage.data(), b->job.stage_bytes);
    QRT_HIP(hipHostMalloc(reinterpret_cast<void **>(&b->h_out), size_t(count) * sizeof(qk::FinalRes), 0),
            "hipHostMalloc");
    // Capture: upload, kernels, download.  No memset nodes: the table kernel
    // clears the work-item counter.
    QRT_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    qubo_status_t cst = QUBO_OK;
    e = hipMemcpyAsync(b->d_mem, b->h_stage, b->job.stage_bytes, hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) cst = qrt::device_error("capture H2D", e);
    if (cst == QUBO_OK) cst = qrt::job_enqueue_kernels(b->job, b->stream, nullptr, nullptr);
    if (cst == QUBO_OK) {
        e = hipMemcpyAsync(b->h_out, b->job.d_out, size_t(count) * sizeof(qk::FinalRes),
                           hipMemcpyDeviceToHost, b->stream);
        if (e != hipSuccess) cst = qrt::device_error("capture D2H", e);
    }
    hipError_t ee = hipStreamEndCapture(b->stream, &b->graph);
    if (cst != QUBO_OK) return cst;
    if (ee != hipSuccess) return qrt::device_error("hipStreamEndCapture", ee);
    QRT_HIP(hipGraphInstantiateWithFlags(&b->exec, b->graph, 0), "hipGraphInstantiate");
    return QUBO_OK;
}

}  // namespace

extern "C" {

qubo_status_t qubo_batch_create(int count, const void *const *Q, const int *n,
                                const qubo_dtype_t *dtype, const qubo_options_t *opt,
                                qubo_batch_t **batch)
{
    try {
        qrt::set_error("");
        if (count < 1 || !Q || !n || !dtype || !batch) {
            qrt::set_error("bad batch arguments");
            return QUBO_EINVAL;
        }
        qubo_batch *b = new qubo_batch();
        qubo_status_t st = batch_build(b, count, Q, n, dtype, opt);
        if (st != QUBO_OK) {
            const std::string keep = qrt::last_error_cstr();
            batch_free(b);
            qrt::set_error(keep);
            return st;
        }
        *batch = b;
        return QUBO_OK;
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

qubo_status_t qubo_batch_run(qubo_batch_t *b, void *hip_stream)
{
    if (!b) {
        qrt::set_error("null batch");
        return QUBO_EINVAL;
    }
    qrt::set_error("");
    hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : b->stream;
    QRT_HIP(hipEventRecord(b->ev0, s), "hipEventRecord");
    QRT_HIP(hipGraphLaunch(b->exec, s), "hipGraphLaunch");
    QRT_HIP(hipEventRecord(b->ev1, s), "hipEventRecord");
    QRT_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    QRT_HIP(hipEventElapsedTime(&b->last_ms, b->ev0, b->ev1), "hipEventElapsedTime");
    b->ran = true;
    return QUBO_OK;
}

qubo_status_t qubo_batch_results(qubo_batch_t *b, qubo_result_t *out)
{
    if (!b || !out) {
        qrt::set_error("null argument");
        return QUBO_EINVAL;
    }
    if (!b->ran) {
        qrt::set_error("batch has not run");
        return QUBO_EINVAL;
    }
    const int count = int(b->order.size());
    for (int w = 0; w < count; w++) {
        qubo_result_t r;
        qubo_status_t st = qrt::job_result(b->job, w, b->h_out[w], &r);
        if (st != QUBO_OK) return st;
        r.kernel_ms = b->last_ms;
        r.total_ms = b->last_ms;
        out[b->order[size_t(w)]] = r;
    }
    return QUBO_OK;
}

qubo_status_t qubo_batch_stats(qubo_batch_t *b, double *states, double *kernel_ms)
{
    if (!b) {
        qrt::set_error("null batch");
        return QUBO_EINVAL;
    }
    if (states) *states = b->job.states;
    if (kernel_ms) *kernel_ms = b->last_ms;
    return QUBO_OK;
}

void qubo_batch_destroy(qubo_batch_t *b) { batch_free(b); }

qubo_status_t qubo_solve_batch(int count, const void *const *Q, const int *n,
                               const qubo_dtype_t *dtype, qubo_result_t *out)
{
    if (!out) {
        qrt::set_error("null output");
        return QUBO_EINVAL;
    }
    qubo_batch_t *b = nullptr;
    qubo_status_t st = qubo_batch_create(count, Q, n, dtype, nullptr, &b);
    if (st != QUBO_OK) return st;
    st = qubo_batch_run(b, nullptr);
    if (st == QUBO_OK) st = qubo_batch_results(b, out);
    const std::string keep = qrt::last_error_cstr();
    qubo_batch_destroy(b);
    qrt::set_error(keep);
    return st;
}

}  // extern "C"

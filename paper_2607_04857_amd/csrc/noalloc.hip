// noalloc.hip -- the allocation-free single solve (qubo_solve_noalloc).
//
// Same plan, kernels and result as qubo_solve with k = 1, but the job's
// device image (descriptors, folded T, float32 Q, M_int / E_s / couplings,
// bound tables, item records, results) lives in one file-scope device
// array instead of a per-call allocation.  Each device holds its own copy of
// the array at its own address, found once per device with
// hipGetSymbolAddress; host code passes that address, never the array's
// name, to copies and kernels.  Everything the kernels read before writing
// is uploaded by this call (the staging image) or cleared by the table
// kernel (item counters, the shared best), so stale contents of a previous
// call never leak into the next one.
#include <array>
#include <chrono>
#include <cstring>
#include <mutex>

#include "runtime.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    bool ready = false;
    void *ptr = nullptr;           // device address of `scratch` on this device
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // walk timing, made once per device
};

std::mutex g_mu;
std::array<DeviceScratch, kMaxDevices> g_dev;

// Set-up on the first call on a device (that device is current).
qubo_status_t scratch_for_device(int dev, DeviceScratch **out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        qrt::set_error("device ordinal beyond the allocation-free table");
        return QUBO_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceScratch &d = g_dev[size_t(dev)];
    if (!d.ready) {
        void *p = nullptr;
        QRT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) {
            qrt::set_error("hipGetSymbolAddress(scratch) returned a null address");
            return QUBO_EDEVICE;
        }
        QRT_HIP(hipEventCreate(&d.ev0), "hipEventCreate");
        QRT_HIP(hipEventCreate(&d.ev1), "hipEventCreate");
        d.ptr = p;
        d.ready = true;
    }
    *out = &d;
    return QUBO_OK;
}

qubo_status_t solve_noalloc(const void *Q, int n, qubo_dtype_t dtype, hipStream_t stream,
                            qubo_result_t *out)
{
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    if (!Q || !out) {
        qrt::set_error("null argument");
        return QUBO_EINVAL;
    }
    int dev = 0;
    QRT_HIP(hipGetDevice(&dev), "hipGetDevice");
    DeviceScratch *ds = nullptr;
    qubo_status_t st = scratch_for_device(dev, &ds);
    if (st != QUBO_OK) return st;
    qrt::tune_autoload();
    qrt::Job job;
    job.plans.resize(1);
    std::string msg;
    st = qplan::make_plan(Q, n, dtype, nullptr, &job.plans[0], &msg);
    if (st != QUBO_OK) {
        qrt::set_error(msg);
        return st;
    }
    job.qf.push_back(dtype == QUBO_FP32 ? static_cast<const float *>(Q) : nullptr);
    st = qrt::job_layout(&job, 0);
    if (st != QUBO_OK) return st;
    if (job.bytes > kScratchBytes) {
        qrt::set_error("qubo_solve_noalloc: the plan needs " + std::to_string(job.bytes) +
                       " bytes of device memory, beyond the " + std::to_string(kScratchBytes) +
                       "-byte scratch array (use qubo_solve)");
        return QUBO_ENOMEM;
    }
    if ((st = qrt::job_bind(&job, ds->ptr)) != QUBO_OK) return st;
    qk::FinalRes fr{};
    do {
        hipError_t e = hipMemcpyAsync(ds->ptr, job.stage.data(), job.stage_bytes,
                                      hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) {
            st = qrt::device_error("hipMemcpyAsync H2D", e);
            break;
        }
        if ((st = qrt::job_enqueue_kernels(job, stream, ds->ev0, ds->ev1)) != QUBO_OK) break;
        e = hipMemcpyAsync(&fr, job.d_out, sizeof(fr), hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) st = qrt::device_error("hipMemcpyAsync D2H", e);
    } while (false);
    // whatever was enqueued finishes before the scratch (and fr) can be reused
    const hipError_t es = hipStreamSynchronize(stream);
    if (st != QUBO_OK) return st;
    if (es != hipSuccess) return qrt::device_error("hipStreamSynchronize", es);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ds->ev0, ds->ev1);
    st = qrt::job_result(job, 0, fr, out);
    if (st != QUBO_OK) return st;
    out->kernel_ms = ms;
    out->total_ms = std::chrono::duration<double, std::milli>(clock::now() - t0).count();
    return QUBO_OK;
}

}  // namespace

extern "C" {

size_t qubo_noalloc_scratch_bytes(void) { return kScratchBytes; }

qubo_status_t qubo_solve_noalloc(const void *Q, int n, qubo_dtype_t dtype, void *hip_stream,
                                 qubo_result_t *out)
{
    try {
        qrt::set_error("");
        return solve_noalloc(Q, n, dtype, static_cast<hipStream_t>(hip_stream), out);
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

}  // extern "C"

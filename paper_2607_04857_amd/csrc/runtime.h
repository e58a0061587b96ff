// runtime.h -- device jobs shared by the single, batch and serving paths.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "kernels.h"
#include "plan.h"

namespace qrt {

void set_error(const std::string &msg);
const char *last_error_cstr();

// HIP call failed: record "what: hipErrorString" and return QUBO_EDEVICE.
qubo_status_t device_error(const char *what, hipError_t e);

#define QRT_HIP(call, what)                                   \
    do {                                                      \
        hipError_t qrt_e_ = (call);                           \
        if (qrt_e_ != hipSuccess) return qrt::device_error(what, qrt_e_); \
    } while (0)

struct DeviceInfo {
    int device = 0;
    int cus = 0;
};
qubo_status_t device_info(DeviceInfo *info);

// Consecutive walked instances sharing one walk kernel variant: one
// persistent launch with its own item numbering and counter.
struct WalkGroup {
    int first = 0, count = 0;            // instance range in the job
    int mcols = 0, vgpr_levels = 0, tier = 0;
    uint64_t items = 0;
    int waves = 0;
};

// A set of planned instances laid out in one device allocation.  Walked
// instances of one variant must be contiguous (callers sort by variant).
struct Job {
    std::vector<qplan::Plan> plans;
    std::vector<const float *> qf;       // caller's fp32 Q per instance (host) or null
    std::vector<WalkGroup> groups;
    int max_A = 0;
    uint64_t total_items = 0;
    double states = 0.0;                 // sum of 2^n

    // device allocation and its host staging image
    void *d_mem = nullptr;
    size_t bytes = 0;
    size_t stage_bytes = 0;              // leading part of d_mem uploaded from the host
    std::vector<unsigned char> stage;    // insts | T... | Qf... (pinned copy in Batch)
    qk::Inst *d_insts = nullptr;
    unsigned long long *d_counter = nullptr;   // one per group
    qk::ItemRes *d_res = nullptr;
    qk::FinalRes *d_out = nullptr;
    int32_t *d_k = nullptr;              // all K tables, instance i at i * kKTable

    // a lone instance whose Q is in device memory (qubo_solve_device): the
    // prepare kernel folds and scales it into T on the device
    const void *dq = nullptr;
    qk::PrepOut *d_prep = nullptr;
    int32_t *d_T0 = nullptr;             // instance 0's T

    // top-k (k > 1): one instance, walked at tier 3
    int topk = 0;
    qk::TopkBufs tkb{};
    qk::Inst h_inst0{};                  // host copy of the descriptor
};

// Lay out plans (already made) into a Job; `waves_per_cu` 0 = occupancy.
qubo_status_t job_layout(Job *job, int waves_per_cu);

// Point the job at device allocation d_mem (job.bytes long) and fill the
// host staging image (instance descriptors, T and float32 Q).
qubo_status_t job_bind(Job *job, void *d_mem);

// Enqueue tables -> walk (one launch per group) -> finish on `stream` (device
// memory must exist and the staging image must already be uploaded).
// Optional events bracket the walk launches.
qubo_status_t job_enqueue_kernels(const Job &job, hipStream_t stream, hipEvent_t walk_begin,
                                  hipEvent_t walk_end);

// Whether two plans run the same walk kernel variant.
bool same_variant(const qplan::Plan &a, const qplan::Plan &b);

// Convert the device result of instance i into the ABI struct.
qubo_status_t job_result(const Job &job, int i, const qk::FinalRes &fr, qubo_result_t *out);

// This thread's stream on the current device (created on first use).
hipStream_t thread_stream(qubo_status_t *st);

// Lay out, upload, run and read back a one-instance job on `stream`
// (synchronous); fills kernel_ms (walk events) and total_ms.
qubo_status_t solve_planned(Job &job, hipStream_t stream, int waves_per_cu, qubo_result_t *out,
                            qubo_state_t *topk = nullptr);

// Load the tuning cache named by the QUBO_TUNE_CACHE environment variable,
// once per process (a no-op when unset; a cache made on another device is
// reported on stderr and ignored).
void tune_autoload();

}  // namespace qrt

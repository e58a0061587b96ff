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

// A set of planned instances laid out in one device allocation.
struct Job {
    std::vector<qplan::Plan> plans;
    std::vector<const float *> qf;       // caller's fp32 Q per instance (host) or null
    int mcols = 0, tier = 0, vgpr_levels = 0;   // shared walk variant of the walked instances
    int max_A = 0;
    uint64_t total_items = 0;
    double states = 0.0;                 // sum of 2^n
    int waves = 0;

    // device allocation and its host staging image
    void *d_mem = nullptr;
    size_t bytes = 0;
    size_t stage_bytes = 0;              // leading part of d_mem uploaded from the host
    std::vector<unsigned char> stage;    // insts | T... | Qf... (pinned copy in Batch)
    qk::Inst *d_insts = nullptr;
    unsigned long long *d_counter = nullptr;
    qk::ItemRes *d_res = nullptr;
    qk::FinalRes *d_out = nullptr;
    int32_t *d_k = nullptr;              // all K tables, instance i at i * kKTable
};

// Lay out plans (already made) into a Job; `waves_per_cu` 0 = occupancy.
qubo_status_t job_layout(Job *job, int waves_per_cu);

// Point the job at device allocation d_mem (job.bytes long) and fill the
// host staging image (instance descriptors, T and float32 Q).
qubo_status_t job_bind(Job *job, void *d_mem);

// Enqueue tables -> walk -> finish on `stream` (device memory must exist and
// the staging image must already be uploaded).  Optional events bracket the
// walk kernel.
qubo_status_t job_enqueue_kernels(const Job &job, hipStream_t stream, hipEvent_t walk_begin,
                                  hipEvent_t walk_end);

// Convert the device result of instance i into the ABI struct.
qubo_status_t job_result(const Job &job, int i, const qk::FinalRes &fr, qubo_result_t *out);

}  // namespace qrt

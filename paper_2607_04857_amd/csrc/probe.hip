// probe.hip -- int32 VALU throughput probe (the measured ceiling of the walk).
//
// Each wave keeps 16 independent accumulators and issues 256 vector
// instructions per loop iteration, so no dependency chain limits issue; the
// grid places waves_per_simd waves on every SIMD of the device.  Ops: 0
// v_add_u32; 1 v_min3_i32; 2 v_add_u32 with one s_add_i32 per two vector adds;
// 3 v_add_u32 with one never-taken s_cmp/s_cbranch per 16 vector adds; 4
// v_pk_add_u16; 5 v_pk_min_i16; 6 v_add_u32 over 160 accumulators, whose
// register footprint admits at most 3 waves per SIMD (the walk's occupancy:
// with few registers the dispatcher may place 4 waves on some SIMDs and 2 on
// others when 3 per SIMD are launched); 7 v_add_f32 (scalar float32, the
// add a float walk would use).  Vector instructions x 64 lanes are counted
// (a packed instruction is one lane-operation on two 16-bit halves).
#include <hip/hip_runtime.h>

#include "runtime.h"

namespace {

template <int OP>
__global__ __launch_bounds__(64) void valu_probe_kernel(int iters, int32_t *__restrict__ out)
{
    // accumulators; 256 vector instructions per iteration either way
    constexpr int NA = OP == 6 ? 160 : 16;
    constexpr int NR = OP == 6 ? 1 : 16;
    int32_t a[NA];
#pragma unroll
    for (int k = 0; k < NA; k++)
        a[k] = OP == 7 ? __float_as_int(float(k)) : int32_t(threadIdx.x) * 7 + k;
    const int32_t b = OP == 7 ? __float_as_int(1.0f) : (int32_t(blockIdx.x) | 1);
    const int32_t c = int32_t(threadIdx.x) ^ 5;
    int32_t sc = int32_t(blockIdx.x);   // scalar work for OP 2 and 3 (wave-uniform)
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
#pragma unroll
            for (int k = 0; k < (OP == 6 ? 256 : 16); k++) {
                if constexpr (OP == 1)
                    asm volatile("v_min3_i32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(b), "v"(c));
                else if constexpr (OP == 4)
                    asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                else if constexpr (OP == 5)
                    asm volatile("v_pk_min_i16 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                else if constexpr (OP == 7)
                    asm volatile("v_add_f32 %0, %1, %0" : "+v"(a[k]) : "v"(b));
                else
                    asm volatile("v_add_u32 %0, %1, %0" : "+v"(a[k % NA]) : "v"(b));
                if constexpr (OP == 2)   // one scalar add per two vector adds
                    if (k % 2 == 1) asm volatile("s_add_i32 %0, %0, 3" : "+s"(sc) : : "scc");
            }
            if constexpr (OP == 3)       // a never-taken compare and branch per 16 adds
                asm volatile("s_cmp_eq_u32 %0, 0x7fffffff\n\ts_cbranch_scc1 1f\n1:" : : "s"(sc) : "scc");
        }
    }
    if constexpr (OP == 2) a[0] ^= sc;
    int32_t x = 0;
#pragma unroll
    for (int k = 0; k < NA; k++) x ^= a[k];
    out[blockIdx.x * 64 + threadIdx.x] = x;
}

}  // namespace

extern "C" qubo_status_t qubo_probe_valu(int op, int waves_per_simd, int iters,
                                         double *lane_ops_per_s, double *ms)
{
    qrt::set_error("");
    if (op < 0 || op > 7 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1) {
        qrt::set_error("bad probe arguments");
        return QUBO_EINVAL;
    }
    qrt::DeviceInfo di;
    qubo_status_t st = qrt::device_info(&di);
    if (st != QUBO_OK) return st;
    const int blocks = di.cus * 4 * waves_per_simd;
    int32_t *d_out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    QRT_HIP(hipMalloc(&d_out, size_t(blocks) * 64 * sizeof(int32_t)), "hipMalloc");
    qubo_status_t rs = QUBO_OK;
    float t = 0.f;
    do {
        hipError_t e;
        if ((e = hipStreamCreate(&s)) != hipSuccess || (e = hipEventCreate(&e0)) != hipSuccess ||
            (e = hipEventCreate(&e1)) != hipSuccess) {
            rs = qrt::device_error("probe set-up", e);
            break;
        }
        for (int rep = 0; rep < 2; rep++) {   // first launch warms up clocks and code
            (void)hipEventRecord(e0, s);
            if (op == 0)
                hipLaunchKernelGGL(valu_probe_kernel<0>, dim3(blocks), dim3(64), 0, s, iters, d_out);
            else if (op == 1)
                hipLaunchKernelGGL(valu_probe_kernel<1>, dim3(blocks), dim3(64), 0, s, iters, d_out);
            else if (op == 2)
                hipLaunchKernelGGL(valu_probe_kernel<2>, dim3(blocks), dim3(64), 0, s, iters, d_out);
            else if (op == 3)
                hipLaunchKernelGGL(valu_probe_kernel<3>, dim3(blocks), dim3(64), 0, s, iters, d_out);
            else if (op == 4)
                hipLaunchKernelGGL(valu_probe_kernel<4>, dim3(blocks), dim3(64), 0, s, iters, d_out);
            else if (op == 5)
                hipLaunchKernelGGL(valu_probe_kernel<5>, dim3(blocks), dim3(64), 0, s, iters, d_out);
            else if (op == 6)
                hipLaunchKernelGGL(valu_probe_kernel<6>, dim3(blocks), dim3(64), 0, s, iters, d_out);
            else
                hipLaunchKernelGGL(valu_probe_kernel<7>, dim3(blocks), dim3(64), 0, s, iters, d_out);
            (void)hipEventRecord(e1, s);
        }
        if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess ||
            (e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) {
            rs = qrt::device_error("probe run", e);
            break;
        }
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(d_out);
    if (rs != QUBO_OK) return rs;
    const double ops = double(blocks) * 64.0 * double(iters) * 256.0;
    if (lane_ops_per_s) *lane_ops_per_s = ops / (double(t) * 1e-3);
    if (ms) *ms = t;
    return QUBO_OK;
}

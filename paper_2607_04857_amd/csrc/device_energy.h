// device_energy.h -- exact per-state energies used by the finishing kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qk {

// Energy of U_N row `idx` from the folded upper-triangular T (exact).
__device__ inline int64_t energy_int(const int32_t *T, int n, uint64_t idx)
{
    int64_t E = 0;
    for (int i = 0; i < n; i++) {
        if (!((idx >> (n - 1 - i)) & 1)) continue;
        int64_t rowsum = 0;
        for (int j = i; j < n; j++)
            if ((idx >> (n - 1 - j)) & 1) rowsum += T[i * n + j];
        E += rowsum;
    }
    return E;
}

// E(x) = sum_{i,j} Q_ij x_i x_j in float64 from the caller's float32 Q,
// summed i ascending then j ascending over the set bits.
__device__ inline double energy_f64(const float *Q, int n, uint64_t idx)
{
    double E = 0.0;
    for (int i = 0; i < n; i++) {
        if (!((idx >> (n - 1 - i)) & 1)) continue;
        for (int j = 0; j < n; j++)
            if ((idx >> (n - 1 - j)) & 1) E += double(Q[i * n + j]);
    }
    return E;
}

}  // namespace qk

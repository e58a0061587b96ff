// kcommon.h -- device helpers shared by the solver's kernels (wave
// reductions, compile-time loops, scalar broadcasts).
#pragma once

#include <type_traits>
#include <utility>

#include "device_energy.h"
#include "kernels.h"

namespace qk {

// ---------------------------------------------------------------- helpers

template <int Begin, int End, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (Begin < End) {
        f(std::integral_constant<int, Begin>{});
        static_for<Begin + 1, End>(static_cast<F &&>(f));
    }
}

constexpr int cx_ctz(int v)
{
    int r = 0;
    while (!(v & 1)) {
        v >>= 1;
        r++;
    }
    return r;
}

__device__ __forceinline__ int32_t sread(int32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint64_t sread64(uint64_t v)
{
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int32_t(uint32_t(v))));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int32_t(uint32_t(v >> 32))));
    return (uint64_t(hi) << 32) | lo;
}

// Minimum of E[0..N) with three-input minima (v_min3_i32) level by level:
// ceil((N-1)/2) VALU ops.
template <int N>
__device__ __forceinline__ int32_t tree_min(const int32_t *e)
{
    if constexpr (N == 1) {
        return e[0];
    } else if constexpr (N == 2) {
        return min(e[0], e[1]);
    } else {
        constexpr int G3 = N / 3, R = N % 3;
        int32_t t[G3 + R];
        static_for<0, G3>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            t[g] = min(min(e[3 * g], e[3 * g + 1]), e[3 * g + 2]);
        });
        static_for<0, R>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            t[G3 + r] = e[3 * G3 + r];
        });
        return tree_min<G3 + R>(t);
    }
}

// Minimum of the 2N energies packed in E[0..N) (two biased 16-bit halves per
// word, the tier-4 layout): packed 16-bit minima level by level
// (v_pk_min_u16; the biased halves compare as unsigned), then the smaller
// half, unbiased.
using u16x2 = unsigned short __attribute__((ext_vector_type(2)));
template <int N>
__device__ __forceinline__ u16x2 pk_tree_min(const u16x2 *e)
{
    if constexpr (N == 1) {
        return e[0];
    } else {
        constexpr int H = N / 2;
        u16x2 t[H + N % 2];
        static_for<0, H>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            t[g] = __builtin_elementwise_min(e[2 * g], e[2 * g + 1]);
        });
        if constexpr (N % 2) t[H] = e[N - 1];
        return pk_tree_min<H + N % 2>(t);
    }
}
template <int N>
__device__ __forceinline__ int32_t tree_min_packed(const int32_t *e)
{
    u16x2 w[N];
    static_for<0, N>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        w[j] = __builtin_bit_cast(u16x2, e[j]);
    });
    const uint32_t x = __builtin_bit_cast(uint32_t, pk_tree_min<N>(w));
    return int32_t(min(x & 0xffffu, x >> 16)) - kPackBias;
}

// Wave-wide minimum: DPP butterflies inside each row of 16 lanes, then the
// four row results through the scalar unit.
__device__ __forceinline__ int32_t wave_min(int32_t v)
{
    constexpr int32_t I = INT32_MAX;
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x124, 0xF, 0xF, false));  // row_ror:4
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x128, 0xF, 0xF, false));  // row_ror:8
    const int32_t a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const int32_t c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return min(min(a, b), min(c, d));
}

// Global (address space 1) view of a table pointer: loads then take a
// uniform base in SGPRs and a lane offset, instead of 64-bit flat addresses.
using gint32 = __attribute__((address_space(1))) const int32_t;
__device__ __forceinline__ const gint32 *to_global(const int32_t *p)
{
    return (const gint32 *)p;
}

// Keeps every element of a chunk vector materialised at this point: the
// walk updates the chunk energies once per state (Eq. incremental_update)
// even where no test reads them, rather than letting the compiler fold
// several flips into their net change.
template <int MC>
__device__ __forceinline__ void pin_vec(int32_t (&e)[MC])
{
#pragma unroll
    for (int j = 0; j < MC; j++) asm("" : "+v"(e[j]));
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ void lexmin(int64_t &bE, uint64_t &bI, int64_t e, uint64_t i)
{
    if (e < bE || (e == bE && i < bI)) {
        bE = e;
        bI = i;
    }
}

// Greedy single-flip descent of the calling wave from start state `start`
// (all-zero for start 0, a hashed state otherwise).  Lane l holds variable l
// (n <= 60 < 64) and its field f_l = T_ll + the couplings with the set
// variables, so flipping l changes E by +-f_l; the largest decrease is taken
// (lowest lane on ties) until no flip lowers E.  Returns the local minimum's
// energy in E_out and its variables (bit l = variable l) in xm_out, the same
// in every lane.
__device__ inline void greedy_descent(const int32_t *T, int n, uint32_t start, int32_t &E_out,
                                      uint64_t &xm_out)
{
    const int lane = int(threadIdx.x) % kWave;
    uint32_t h = start * 0x9E3779B9u + uint32_t(lane) * 0x85EBCA6Bu;
    h ^= h >> 15;
    h *= 0xC2B2AE35u;
    h ^= h >> 13;
    int x = (start != 0 && lane < n) ? int(h & 1u) : 0;
    const uint64_t xm = __builtin_amdgcn_ballot_w64(x != 0);
    int32_t f = 0, own = 0;   // field; sum of row l over the set j >= l
    if (lane < n) {
        f = T[lane * n + lane];
        own = x ? T[lane * n + lane] : 0;
        for (int j = 0; j < n; j++) {
            if (j == lane || !((xm >> j) & 1)) continue;
            const int32_t c = j < lane ? T[j * n + lane] : T[lane * n + j];
            f += c;
            if (x && j > lane) own += c;
        }
    }
    int32_t E = int32_t(wave_sum64(own));
    for (int it = 0; it < 4 * n; it++) {
        const int32_t gain = lane < n ? (x ? -f : f) : INT32_MAX;
        // smallest gain (DPP minimum), lowest lane on ties
        const int32_t g = wave_min(gain);
        if (g >= 0) break;
        const int k = int(__builtin_ctzll(__builtin_amdgcn_ballot_w64(gain == g)));
        const int32_t sgn = __shfl(x, k, kWave) ? -1 : 1;   // 1 -> 0 subtracts couplings
        E += g;
        if (lane == k) x ^= 1;
        else if (lane < n) f += sgn * (k < lane ? T[k * n + lane] : T[lane * n + k]);
    }
    E_out = E;
    xm_out = __builtin_amdgcn_ballot_w64(x != 0);
}

}  // namespace qk

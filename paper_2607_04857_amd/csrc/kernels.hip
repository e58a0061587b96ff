// kernels.hip -- gfx950 kernels of the exhaustive dense-QUBO solver.
//
// Method (paper Sec. II-III): split every state x = [x_p | x_s] into an
// A-bit prefix and a B-bit suffix.  For a fixed prefix the energies of all
// 2^B states of its chunk are (Sec. II-C, Eq. chunk_energy_final)
//     E(C_xp) = E_p(x_p) 1 + x_p M_int + E_s(U_B),   M_int = Q_ps U_B^T.
// Walking the prefixes in reflected Gray order (Sec. III-B) changes x_p by one
// bit k per step, so the suffix-dependent vector E_sd = x_p M_int + E_s moves
// by +-M_int[k] (Eq. incremental_update): one int32 add per state.
//
// MI355X mapping:
//  * one wavefront owns all 2^B columns of its chunk: lane l holds columns
//    s = j*64 + l (j < MC), i.e. E_sd lives in MC VGPRs per lane (column-wise
//    split, Sec. III-C.2, at lane granularity);
//  * the rows M_int[k] of the most frequently flipped Gray levels stay on
//    chip: by default levels 0-2 and 5 in VGPRs and 3-4 in LDS (8 KB per
//    wave), which fits 128 VGPRs and so four waves per SIMD; other variants
//    keep 5, 6, 8 or 12 levels in VGPRs; higher levels are read from L2 when
//    they flip (level 6 once per 128 steps; level 5, in the 5-level variants,
//    once per 64);
//  * wavefronts take work items (2^L consecutive Gray steps of the prefix,
//    the "straightforward" split of Sec. III-C.1 along the Gray index) from an
//    atomic counter, one at a time; the grid is persistent;
//  * the scalar unit keeps the prefix self-energy E_p: the walk is unrolled
//    over 64-step super-blocks in which the five lowest Gray levels follow a
//    static pattern and level 5 flips once, in the middle, so the flip
//    sequence is known at compile time and E_p of each low pattern follows
//    from SGPR fields refreshed only when a higher prefix bit flips;
//  * the candidate test "min over the chunk + E_p <= best" is, by default
//    (tier 2), a lower bound from one DPP wave minimum per super-block and a
//    per-offset table, tested against a cheap upper bound of the thresholds
//    once per 16 steps; exact per-step tests run only when that passes (tier
//    1 does the exact v_min3 test at every step).  Each step still updates
//    the chunk vector once (pinned, so the compiler cannot fold flips).  Ties
//    resolve to the lowest prefix row here and to the lowest suffix in the
//    final rescan, giving the lowest U_N index overall.
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

// ---------------------------------------------------------------- tables

// Greedy single-flip descent from two starts per wave (the all-zero state
// for wave 0's first start, hashed states otherwise), lowering the
// instance's shared best to the energy of the local minima found.  Any
// state's energy is a valid threshold for the walk (the state's own chunk
// still passes it), and a local minimum of a dense QUBO is usually close to
// the global one, so walk waves start with a near-final threshold.  Lane l
// holds variable l (n <= 60 < 64) and its field f_l = T_ll + sum of the
// couplings with the set variables: flipping l changes E by +-f_l.
__device__ void seed_best(const Inst &I, int wave)
{
    const int n = I.n, lane = int(threadIdx.x) % kWave;
    const int32_t *T = I.T;
    int32_t bestE = kNoEnergy;
    for (int rep = 0; rep < 2; rep++) {
        const uint32_t start = uint32_t(wave) * 2u + uint32_t(rep);
        uint32_t h = start * 0x9E3779B9u + uint32_t(lane) * 0x85EBCA6Bu;
        h ^= h >> 15;
        h *= 0xC2B2AE35u;
        h ^= h >> 13;
        int x = (start != 0 && lane < n) ? int(h & 1u) : 0;
        uint64_t xm = __builtin_amdgcn_ballot_w64(x != 0);
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
        bestE = min(bestE, E);
    }
    if (lane == 0) atomicMin(I.gbest, bestE);
}

__global__ __launch_bounds__(256) void tables_kernel(const Inst *__restrict__ insts,
                                                     unsigned long long *__restrict__ counters,
                                                     int n_counters)
{
    const Inst I = insts[blockIdx.y];
    if (blockIdx.x == 0 && blockIdx.y == 0)
        for (int c = int(threadIdx.x); c < n_counters; c += int(blockDim.x)) counters[c] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0 && I.gbest) {
        atomicExch(I.gbest, kNoEnergy);
        __threadfence();
    }
    if (I.bits) {   // no item has reported yet
        const uint64_t words = (I.n_items + 31) / 32;
        for (uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < words;
             w += uint64_t(gridDim.x) * blockDim.x)
            I.bits[w] = 0u;
    }
    if (I.direct) return;
    const int n = I.n, A = I.A, B = I.B;
    const uint32_t NS = 1u << B;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    const int32_t *T = I.T;
    // M_int[v][s] = sum over the set suffix bits t of s of T[v][A + t]
    // (Sec. II-C; bit t of the suffix row is (s >> (B-1-t)) & 1), as the sum
    // of two partial sums built first in LDS: part[v][s & 31] over the five
    // lowest bits of s and part[v][32 + (s >> 5)] over the others.
    __shared__ int32_t part[kMaxPrefixRows][64];
    for (uint32_t e = threadIdx.x; e < uint32_t(A) * 64u; e += blockDim.x) {
        const int v = int(e / 64u), x = int(e % 64u);
        int32_t acc = 0;
        if (x < 32) {
            for (int u = 0; u < 5; u++)
                if ((x >> u) & 1) acc += T[v * n + A + B - 1 - u];
        } else {
            const int hi = x - 32;
            for (int u = 0; u < B - 5; u++)
                if ((hi >> u) & 1) acc += T[v * n + A + B - 6 - u];
        }
        part[v][x] = acc;
    }
    __syncthreads();
    // rows A..2A-1 hold -M_int: a flip whose direction is known only at
    // run time then adds one row or the other, without a branch
    for (uint32_t e = tid; e < uint32_t(A) * NS; e += stride) {
        const int v = int(e >> B);
        const uint32_t s = e & (NS - 1);
        const int32_t m = part[v][s & 31u] + part[v][32u + (s >> 5)];
        I.M[e] = m;
        I.M[uint32_t(A) * NS + e] = -m;
    }
    // E_s(U_B)[s] = sum_{t <= u, both set} T[A+t][A+u] (Sec. III-A, step 2)
    for (uint32_t s = tid; s < NS; s += stride) {
        int32_t acc = 0;
        for (int t = 0; t < B; t++) {
            if (!((s >> (B - 1 - t)) & 1u)) continue;
            for (int u = t; u < B; u++)
                if ((s >> (B - 1 - u)) & 1u) acc += T[(A + t) * n + A + u];
        }
        I.EB[s] = acc;
    }
    // prefix couplings, one lane per variable
    for (uint32_t e = tid; e < uint32_t(A) * kWave; e += stride) {
        const int w = int(e / kWave), l = int(e % kWave);
        int32_t v = 0;
        if (l < A && l != w) v = (l < w) ? T[l * n + w] : T[w * n + l];
        I.S[e] = v;
        I.S[uint32_t(A) * kWave + e] = -v;   // negated rows, as for M_int
    }
    if (blockIdx.x != 0) return;
    __syncthreads();
    // (only when the walk covers every state: a restricted item range must
    // not start from an energy found outside it)
    if (I.gbest && I.item_local0 == 0 && I.n_items == (uint64_t(1) << (A - I.L)))
        seed_best(I, int(threadIdx.x) / kWave);
    for (uint32_t e = threadIdx.x; e < uint32_t(A) * kLowLevels; e += blockDim.x) {
        const int w = int(e / kLowLevels), t = int(e % kLowLevels), l = A - 1 - t;
        int32_t v = 0;
        if (l != w) v = (l < w) ? T[l * n + w] : T[w * n + l];
        I.K[kKBound + e] = v;
    }
    // Tier-2 bound constants.  Inside a 64-step super-block the five lowest
    // Gray levels follow the static pattern p(o) = g(o) & 31 from 0, and the
    // level-5 bit moves once (by cm = +-1) at o = 32, so
    //   E_sd(o) - E_sd(0) = sum_{t<5} p_t(o) M[A-1-t] + [o >= 32] cm M[A-6].
    // D = its minimum over all 2^B columns, a lower bound of how far the
    // chunk minimum can fall from its value at the super-block start.
    // All 96 (table, offset) minima at once: per-thread minima over the
    // thread's columns, wave minima by shuffles, one exchange through LDS.
    constexpr int NQ = 3 * kPatterns;
    __shared__ int32_t red[256 / kWave][NQ];
    __shared__ int32_t c2s[NQ];
    int32_t mcol[4][kLowLevels + 1];   // M rows of levels 0..kLowLevels at this thread's columns
    for (int k = 0; k < 4; k++) {
        const uint32_t col = threadIdx.x + 256u * uint32_t(k);
        for (int t = 0; t <= kLowLevels; t++)
            mcol[k][t] = col < NS ? part[A - 1 - t][col & 31u] + part[A - 1 - t][32u + (col >> 5)] : 0;
    }
    const int wl = int(threadIdx.x) % kWave, wv = int(threadIdx.x) / kWave;
    for (int q = 0; q < NQ; q++) {
        const int tab = q / kPatterns, oo = q % kPatterns;
        const int cm = tab == 0 ? 0 : (tab == 1 ? 1 : -1);
        const int o = tab == 0 ? oo : kPatterns + oo;
        const int pat = (o ^ (o >> 1)) & (kPatterns - 1);
        int32_t mn = INT32_MAX;
        for (int k = 0; k < 4; k++) {
            if (threadIdx.x + 256u * uint32_t(k) >= NS) continue;
            int32_t v = cm * mcol[k][kLowLevels];
            for (int t = 0; t < kLowLevels; t++)
                if ((pat >> t) & 1) v += mcol[k][t];
            mn = min(mn, v);
        }
        mn = wave_min(mn);
        if (wl == 0) red[wv][q] = mn;
    }
    __syncthreads();
    if (int(threadIdx.x) < NQ) {
        const int q = int(threadIdx.x), tab = q / kPatterns, oo = q % kPatterns;
        const int o = tab == 0 ? oo : kPatterns + oo;
        const int pat = (o ^ (o >> 1)) & (kPatterns - 1);
        int32_t d = red[0][q];
        for (int w = 1; w < 256 / kWave; w++) d = min(d, red[w][q]);
        int32_t elow = 0;   // couplings among the set low variables
        for (int t = 0; t < kLowLevels; t++)
            for (int u = t + 1; u < kLowLevels; u++)
                if (((pat >> t) & 1) && ((pat >> u) & 1)) elow += T[(A - 1 - u) * n + (A - 1 - t)];
        I.K[(3 + tab) * kPatterns + oo] = d;
        I.K[tab * kPatterns + oo] = elow + d;
        c2s[q] = elow + d;
    }
    __syncthreads();
    if (threadIdx.x < 6) {   // min of C2 over each 16-step segment of each table
        const int tab = int(threadIdx.x) / 2, sg = int(threadIdx.x) % 2;
        int32_t m = INT32_MAX;
        for (int oo = sg * kSegSteps; oo < (sg + 1) * kSegSteps; oo++) m = min(m, c2s[tab * kPatterns + oo]);
        I.K[kKC2Min + threadIdx.x] = m;
    }
    if (threadIdx.x == 6 || threadIdx.x == 7) I.K[kKC2Min + threadIdx.x] = 0;
}

// ---------------------------------------------------------------- walk

// Wave-wide minimum for the tier-2 super-block base: DPP inside each row of
// 16 lanes, then row broadcasts, result in lane 63.
__device__ __forceinline__ int32_t wave_min_bcast(int32_t v)
{
    // lanes a DPP source leaves unwritten read INT32_MAX, the identity of min
    constexpr int32_t I = INT32_MAX;
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x124, 0xF, 0xF, false));  // row_ror:4
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x128, 0xF, 0xF, false));  // row_ror:8
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = min(v, __builtin_amdgcn_update_dpp(I, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// TIER 1: the chunk minimum (v_min3 tree) is compared with the threshold at
//         every Gray step.
// TIER 2: each lane takes its chunk minimum lm0 once per 64-step
//         super-block; at offset o the chunk minimum is at least
//         W0 + D(o) (table K), W0 the wave minimum of lm0, so step o needs
//         only the scalar test W0 <= THR - D(o).  Each 16-step segment first
//         tests lm0 against an upper bound of its 16 thresholds (one vector
//         compare); only when a lane passes are W0 and the exact thresholds
//         formed and tested.
// Resident waves per SIMD each variant is register-allocated for: the full
// 12-level row cache fits 256 VGPRs (2 waves); the 8- and 6-level caches
// leave room for a third (MC=16) or a fourth (MC=8) wave.
// LR: the rows of Gray levels 3 and 4 live in LDS (2 x MC x 64 dwords per
// wave) instead of VGPRs, which leaves room for a fourth wave per SIMD.
template <int MC, int G, bool LR = false>
constexpr int walk_waves_per_simd()
{
    return LR ? 4 : (G >= 12 ? (MC >= 16 ? 2 : (MC >= 8 ? 3 : 4)) : (G <= 5 ? 4 : (MC >= 16 ? 3 : 4)));
}
// (G = 6 and 8 with MC = 16 target 3 waves, G = 5 four; 8 and 5 spill a few
// values outside the unrolled steps.)

// Bytes of dynamic LDS ahead of the LDS rows (the tier-3 list), 16-aligned.
__host__ __device__ inline size_t lds_rows_offset(int tier, int k)
{
    (void)k;
    return tier == 3 ? (topk_lds_bytes() + 15) & ~size_t(15) : 0;
}
template <int MC>
constexpr size_t lds_rows_bytes()
{
    return size_t(2) * MC * kWave * sizeof(int32_t);
}

// ---- tier-3 list (top-k).  One wave per workgroup.  The list's scalars
// live in dynamic LDS (kTopkMetaWords 64-bit words); its k entries (E and
// prefix row) live in global memory, at listE / listR + blockIdx.x * k, and
// entry p is written and read only by lane p % 64, so each lane reads its own
// earlier writes in program order and no fence is needed.  Only the rare
// candidate path touches the entries (from L2), and the LDS stays free for
// the row cache, so tier 3 runs the LDS row-cache variants at four waves per
// SIMD whatever k is.  No list state is held in registers and the list code
// sits in functions that are not inlined: the walk's registers stay those of
// tier 2.
//   M[0] entries used  M[1] slot of the largest key  M[2] its E (kNoEnergy
//   until the list is full)  M[3] lowest shared bound seen  M[4] k
//   M[5] histogram bin shift
//   P[0] the largest key's row  P[1] gthr  P[2] listE  P[3] listR
//   P[4] listCount  P[5] hist  P[6] lowbin  P[7] hist_lo
//   (M = words 0..3 as int32, P = words 4..12)
//
// Shared bound.  Every key that enters any wave's list is also counted in a
// device-wide histogram by energy bin.  Keys entered belong to distinct
// chunks (each chunk is walked once), so if the bins up to b hold at least k
// of them, at least k chunks have a key <= the upper edge of bin b, which
// therefore bounds the instance's k-th smallest chunk key: no chunk above it
// can be among the k smallest.  Each insertion recomputes that edge and
// lowers gthr; every wave's threshold is min(its own list's largest E when
// full, gthr).
extern __shared__ uint64_t tk_lds[];

__device__ __forceinline__ int32_t *tk_M() { return reinterpret_cast<int32_t *>(tk_lds); }
__device__ __forceinline__ uint64_t *tk_P() { return tk_lds + 4; }
// this wave's k list entries in global memory
__device__ __forceinline__ int32_t *tk_E(int k)
{
    return reinterpret_cast<int32_t *>(sread64(tk_P()[2])) + size_t(blockIdx.x) * size_t(k);
}
__device__ __forceinline__ uint64_t *tk_R(int k)
{
    return reinterpret_cast<uint64_t *>(sread64(tk_P()[3])) + size_t(blockIdx.x) * size_t(k);
}
__device__ __forceinline__ int32_t *tk_gthr()
{
    return reinterpret_cast<int32_t *>(sread64(tk_P()[1]));
}

__device__ __forceinline__ void tk_init(const TopkWalk &tk)
{
    if (threadIdx.x == 0) {
        int32_t *M = tk_M();
        uint64_t *P = tk_P();
        M[0] = 0;
        M[1] = 0;
        M[2] = kNoEnergy;
        M[3] = kNoEnergy;
        M[4] = tk.k;
        M[5] = tk.hist_shift;
        P[0] = 0;
        P[1] = reinterpret_cast<uint64_t>(tk.gthr);
        P[2] = reinterpret_cast<uint64_t>(tk.listE);
        P[3] = reinterpret_cast<uint64_t>(tk.listR);
        P[4] = reinterpret_cast<uint64_t>(tk.listCount);
        P[5] = reinterpret_cast<uint64_t>(tk.hist);
        P[6] = reinterpret_cast<uint64_t>(tk.lowbin);
        P[7] = uint64_t(tk.hist_lo);
    }
    __syncthreads();
}

// Threshold at an item start: min(largest E of the full list, shared bound).
__device__ __noinline__ int32_t tk_threshold()
{
    int32_t *M = tk_M();
    const int32_t g = sread(__hip_atomic_load(tk_gthr(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const int32_t gm = min(sread(M[3]), g);
    const int32_t t = min(sread(M[2]), gm);
    __syncthreads();
    if (threadIdx.x == 0) M[3] = gm;
    __syncthreads();
    return t;
}

// Largest key (E, row) of the full list: store it and its slot, publish its
// E to the shared bound; returns that E.
__device__ int32_t tk_rescan(int k)
{
    __syncthreads();              // lane 0's LDS scalar stores are visible to the wave
    const int lane = int(threadIdx.x);
    const int32_t *E = tk_E(k);
    const uint64_t *R = tk_R(k);
    int32_t mE = INT32_MIN;
    uint64_t mR = 0;
    int mP = 0;
    for (int p = lane; p < k; p += kWave) {
        const int32_t e = E[p];
        const uint64_t r = R[p];
        if (e > mE || (e == mE && r > mR)) {
            mE = e;
            mR = r;
            mP = p;
        }
    }
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        const int32_t oE = __shfl_xor(mE, off, kWave);
        const uint64_t oR = __shfl_xor(mR, off, kWave);
        const int oP = __shfl_xor(mP, off, kWave);
        if (oE > mE || (oE == mE && oR > mR)) {
            mE = oE;
            mR = oR;
            mP = oP;
        }
    }
    mE = sread(mE);
    if (lane == 0) {
        int32_t *M = tk_M();
        M[1] = mP;
        M[2] = mE;
        M[3] = min(M[3], mE);
        tk_P()[0] = mR;
        atomicMin(tk_gthr(), mE);
    }
    return mE;
}

// Count key energy Ec in the shared histogram and lower gthr to the upper
// edge of the first bin where the running count reaches k.
__device__ void tk_count(int32_t Ec, int k)
{
    const uint64_t *P = tk_P();
    uint32_t *hist = reinterpret_cast<uint32_t *>(sread64(P[5]));
    int32_t *lowbin = reinterpret_cast<int32_t *>(sread64(P[6]));
    const int64_t lo = int64_t(sread64(P[7]));
    const int shift = sread(tk_M()[5]);
    const int lane = int(threadIdx.x);
    int b = int((int64_t(Ec) - lo) >> shift);
    b = b < 0 ? 0 : (b >= kTopkBins ? kTopkBins - 1 : b);
    if (lane == 0) {
        atomicAdd(&hist[b], 1u);
        atomicMin(lowbin, b);
    }
    __threadfence();
    int base = sread(__hip_atomic_load(lowbin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    uint32_t cum = 0;
    for (; base < kTopkBins; base += kWave) {
        const int bin = base + lane;
        uint32_t c = bin < kTopkBins
                         ? __hip_atomic_load(&hist[bin], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                         : 0u;
        // inclusive prefix sum over the wave
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(c, off, kWave);
            if (lane >= off) c += o;
        }
        const uint32_t total = uint32_t(__builtin_amdgcn_readlane(int32_t(c), kWave - 1));
        if (cum + total >= uint32_t(k)) {
            const uint64_t hit = __builtin_amdgcn_ballot_w64(cum + c >= uint32_t(k));
            const int bstar = base + int(__builtin_ctzll(hit));
            const int64_t edge = lo + (int64_t(bstar + 1) << shift) - 1;
            const int32_t T = edge > int64_t(kNoEnergy) ? kNoEnergy : int32_t(edge);
            if (lane == 0) atomicMin(tk_gthr(), T);
            return;
        }
        cum += total;
    }
}

// Offer chunk key (Ec, rc), Ec <= the current threshold: append while the
// list has room, else replace the largest key if (Ec, rc) is smaller.
// Returns the new threshold.
__device__ __noinline__ int32_t tk_insert(int32_t Ec, uint64_t rc)
{
    Ec = sread(Ec);
    rc = sread64(rc);
    int32_t *M = tk_M();
    __syncthreads();
    const int cnt = sread(M[0]);
    const int k = sread(M[4]);
    int32_t lkth = sread(M[2]);
    bool entered = false;
    if (cnt < k) {
        __syncthreads();
        if (int(threadIdx.x) == cnt % kWave) {   // the lane that owns entry cnt
            tk_E(k)[cnt] = Ec;
            tk_R(k)[cnt] = rc;
        }
        if (threadIdx.x == 0) M[0] = cnt + 1;
        entered = true;
        if (cnt + 1 == k) lkth = tk_rescan(k);
    } else {
        const uint64_t lkR = sread64(tk_P()[0]);
        if (Ec < lkth || (Ec == lkth && rc < lkR)) {
            const int pos = sread(M[1]);
            __syncthreads();
            if (int(threadIdx.x) == pos % kWave) {   // the lane that owns entry pos
                tk_E(k)[pos] = Ec;
                tk_R(k)[pos] = rc;
            }
            entered = true;
            lkth = tk_rescan(k);
        }
    }
    if (entered) tk_count(Ec, k);
    const int32_t g = sread(__hip_atomic_load(tk_gthr(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    __syncthreads();
    if (threadIdx.x == 0) M[3] = min(M[3], g);
    __syncthreads();
    return min(lkth, sread(M[3]));
}

// Publish the number of entries of the wave's list (the entries are already
// in listE / listR at slot blockIdx.x * k).
__device__ __noinline__ void tk_flush()
{
    __syncthreads();
    const int32_t *M = tk_M();
    const uint64_t *P = tk_P();
    const int cnt = sread(M[0]);
    if (threadIdx.x == 0) reinterpret_cast<int32_t *>(sread64(P[4]))[blockIdx.x] = cnt;
}

// TIER 3: tier 2's bound test against a top-k threshold instead of the best
//         energy: the wave keeps the k smallest chunk keys it has met in LDS.
template <int MC, int G, int TIER, bool LR = false>
__global__ __launch_bounds__(kWave, (walk_waves_per_simd<MC, G, LR>())) void walk_kernel(
    const Inst *__restrict__ insts, int n_inst, uint64_t total_items,
    unsigned long long *__restrict__ counter, const int32_t *__restrict__ kall, TopkWalk tk)
{
    static_assert(TIER >= 1 && TIER <= 3, "tier");
    static_assert(G >= kLowLevels && G <= kMaxVgprLevels, "VGPR-resident levels");
    constexpr int SEG = kSegSteps;   // steps per segment
    const int lane = int(threadIdx.x);
    const uint32_t ulane = threadIdx.x;
    // row v of a lane-major [rows][MC*64] table: uniform base pointer
    auto trow = [](const gint32 *t, int v) { return t + size_t(v) * (MC * kWave); };
    // LR: rows of levels 3 and 4 after the (tier-3) list in dynamic LDS
    int32_t *const ldsR = reinterpret_cast<int32_t *>(
        reinterpret_cast<char *>(tk_lds) + lds_rows_offset(TIER, tk.k));

    int cur = -1;
    // the tables, addressed as global memory (uniform base + lane offset +
    // immediate), not through generic pointers
    const gint32 *M = nullptr, *EB = nullptr, *S = nullptr;
    int kbase = 0;                // this instance's K table: kall[kbase ...] (scalar loads)
    int A = 0, L = 0;
    uint64_t item_begin = 0, item_local0 = 0;
    int32_t R[G][MC];        // M_int rows of Gray levels 0..G-1 (variable A-1-t)
    int32_t Smid = 0;          // couplings of the middle-level variable, one lane each
    int32_t SmidL[kLowLevels];  // couplings of the middle-level variable with the low ones
    const int32_t *Tm = nullptr;  // the instance's folded T (the diagonal is
    int nT = 0;                   // re-read per item rather than held in a VGPR)
    int32_t CR[kPatterns];   // low-low coupling increments per pattern
    int32_t *gbest = nullptr;     // the current instance's shared best
    int32_t best = kNoEnergy;     // tier 3: the current top-k threshold
    uint64_t bestRow = ~0ull;

    if constexpr (TIER == 3) tk_init(tk);

    for (;;) {
        uint64_t g = 0;
        if (lane == 0) g = atomicAdd(counter, 1ull);
        g = sread64(g);
        if (g >= total_items) break;

        // instance owning item g: first k with item_end > g
        int lo = 0, hi = n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (insts[mid].item_end > g) hi = mid;
            else lo = mid + 1;
        }
        if (lo != cur) {
            cur = lo;
            const Inst &I = insts[lo];
            M = to_global(I.M);
            EB = to_global(I.EB);
            S = to_global(I.S);
            kbase = I.kslot * kKTable;
            A = I.A;
            L = I.L;
            item_begin = I.item_begin;
            item_local0 = I.item_local0;
            static_for<0, G>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                const bool have = t < A;
                const int v = have ? A - 1 - t : 0;
                if constexpr (LR && (t == 3 || t == 4)) {
                    // each lane writes and later reads only its own columns
#pragma unroll
                    for (int j = 0; j < MC; j++)
                        ldsR[(t - 3) * (MC * kWave) + j * kWave + lane] =
                            have ? trow(M, v)[j * kWave + ulane] : 0;
                } else {
#pragma unroll
                    for (int j = 0; j < MC; j++) R[t][j] = have ? trow(M, v)[j * kWave + ulane] : 0;
                }
            });
            Smid = S[size_t(A - 1 - kLowLevels) * kWave + ulane];
            static_for<0, kLowLevels>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                SmidL[t] = kall[kbase + kKBound + (A - 1 - kLowLevels) * kLowLevels + t];
            });
            Tm = I.T;
            nT = I.n;
            // Sll(t,u): coupling of the low variables A-1-t and A-1-u
            int32_t Sll[kLowLevels][kLowLevels];
            static_for<0, kLowLevels>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                static_for<0, kLowLevels>([&](auto uc) {
                    constexpr int u = decltype(uc)::value;
                    // loads through the descriptor's generic pointers count as
                    // divergent; readfirstlane keeps these constants in SGPRs
                    Sll[t][u] = (t == u) ? 0 : sread(S[(A - 1 - u) * kWave + (A - 1 - t)]);
                });
            });
            CR[0] = 0;
            static_for<1, kPatterns>([&](auto pc) {
                constexpr int p = decltype(pc)::value;
                constexpr int t = cx_ctz(p);
                constexpr int pp = p & (p - 1);
                int32_t acc = 0;
                static_for<0, kLowLevels>([&](auto uc) {
                    constexpr int u = decltype(uc)::value;
                    if constexpr ((pp >> u) & 1) acc += Sll[t][u];
                });
                CR[p] = acc;
            });
            best = kNoEnergy;
            bestRow = ~0ull;
            if constexpr (TIER != 3) gbest = I.gbest;
        }

        // Best energy found by any wave for this instance (published at the
        // end of each item): a chunk can improve the final answer only if its
        // key is at most that.  (A chunk tying it with an unknown row is still
        // recorded: bestRow restarts at the largest row whenever the shared
        // value lowers best.)
        if constexpr (TIER != 3) {
            const int32_t g0 = sread(__hip_atomic_load(gbest, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT));
            if (g0 < best) {
                best = g0;
                bestRow = ~0ull;
            }
        }

        // ---- item set-up: state g(i0) from scratch
        const uint64_t qloc = g - item_begin + item_local0;   // the instance's item number
        const uint64_t i0 = qloc << L;
        const uint64_t sb0 = i0 >> kSuperLog;
        const uint64_t sbEnd = sb0 + (1ull << (L - kSuperLog));
        const uint64_t row0 = i0 ^ (i0 >> 1);

        int32_t E[MC];
#pragma unroll
        for (int j = 0; j < MC; j++) E[j] = EB[j * kWave + ulane];
        for (int v = 0; v < A; v++) {
            if ((row0 >> (A - 1 - v)) & 1) {
#pragma unroll
                for (int j = 0; j < MC; j++) E[j] += trow(M, v)[j * kWave + ulane];
            }
        }
        // F: field of every prefix variable from the non-low ones (levels >= 4,
        // variables 0..A-5), plus its diagonal; one lane per variable.
        const int32_t diagl = lane < A ? Tm[lane * nT + lane] : 0;   // T[l][l], lane l < A
        int32_t F = diagl;
        for (int w = 0; w <= A - 1 - kLowLevels; w++)
            if ((row0 >> (A - 1 - w)) & 1) F += S[size_t(w) * kWave + ulane];
        // E_nl = energy of the non-low prefix bits = (sum_set F_w + T_ww) / 2
        const bool lbit = lane <= A - 1 - kLowLevels && ((row0 >> (A - 1 - lane)) & 1);
        int32_t Enl = int32_t(wave_sum64(lbit ? int64_t(F) + diagl : 0) / 2);
        Enl = sread(Enl);
        int32_t H[kLowLevels];
        static_for<0, kLowLevels>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            H[t] = __builtin_amdgcn_readlane(F, A - 1 - t);
        });
        if constexpr (TIER == 3) best = tk_threshold();

        // TIER 1: THR[p] = best - E_p(low pattern p): the chunk holds a
        // candidate when its minimum E_sd is <= THR of the current pattern.
        int32_t THR[kPatterns];
        auto build_thr = [&]() {
            THR[0] = best - Enl;
            static_for<1, kPatterns>([&](auto pc) {
                constexpr int p = decltype(pc)::value;
                constexpr int t = cx_ctz(p);
                constexpr int pp = p & (p - 1);
                THR[p] = THR[pp] - H[t] - CR[p];
            });
        };
        // TIER 2: for the 16 offsets o of segment `seg` (o = 16 seg + o2),
        //   tp(o) = best - E_p(low pattern at o) - C2(o)   (K table tab),
        // computed by walking the Gray sequence of patterns g(o) & 31 from
        // the segment's first one; hs = the sum of H[t] over the set low
        // bits.  f(o2, tp) is called for every offset.  Step o can hold a
        // candidate only if W0 <= tp(o) + D(o) - ELOW(o).
        auto for_each_tp = [&](auto segc, int tab, auto &&f) {
            constexpr int seg = decltype(segc)::value;
            constexpr int o0 = seg * SEG;
            constexpr int p0 = (o0 ^ (o0 >> 1)) & (kPatterns - 1);
            int32_t hs = 0;
            static_for<0, kLowLevels>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                if constexpr ((p0 >> t) & 1) hs += H[t];
            });
            static_for<0, SEG>([&](auto oc) {
                constexpr int o2 = decltype(oc)::value;
                constexpr int o = o0 + o2;
                if constexpr (o2 > 0) {
                    constexpr int pa0 = ((o - 1) ^ ((o - 1) >> 1)) & (kPatterns - 1);
                    constexpr int pa1 = (o ^ (o >> 1)) & (kPatterns - 1);
                    constexpr int t = cx_ctz(pa0 ^ pa1);
                    if constexpr (((pa1 >> t) & 1) != 0) hs += H[t];
                    else hs -= H[t];
                }
                f(oc, (best - Enl) - hs - kall[kbase + tab * kPatterns + (o & (kPatterns - 1))]);
            });
        };
        // Thresholds of the current segment, kept in SGPRs.
        int32_t TP[SEG];
        auto build_tp = [&](auto segc, int tab) {
            for_each_tp(segc, tab, [&](auto oc, int32_t tp) { TP[decltype(oc)::value] = tp; });
        };
        if constexpr (TIER == 1) build_thr();

        // A non-low prefix variable w flips (direction up: 0 -> 1); SLw[t] is
        // its coupling with the low variable A-1-t; Sd is its coupling
        // column with the sign of the flip applied.
        auto nonlow_flip = [&](int w, bool up, int32_t Sd, const int32_t *SLw) {
            const int32_t Fw = __builtin_amdgcn_readlane(F, w);
            Enl = up ? Enl + Fw : Enl - Fw;
            F += Sd;
            static_for<0, kLowLevels>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                H[t] = up ? H[t] + SLw[t] : H[t] - SLw[t];
            });
        };

        int32_t itemE = kNoEnergy;
        uint64_t itemRow = 0;
        int found = 0;
        int32_t W0 = 0;    // TIER 2: exact wave minimum at the super-block start
                           // (taken on the cold path only)
        int32_t lm0 = 0;   // TIER 2: this lane's chunk minimum at the super-block start
        int tab2 = 0;      // TIER 2: K table of the current segment (0 before the middle
                           // flip, 1 / 2 after it with level 5 rising / falling)

        // Candidate test at Gray step i with chunk minimum lm and threshold thr.
        auto candidate = [&](int32_t lm, int32_t thr, uint64_t i) {
            if (__builtin_amdgcn_ballot_w64(lm <= thr)) {
                const int32_t wmin = wave_min(lm);
                const int32_t Ec = wmin + (best - thr);   // + E_p
                const uint64_t rc = i ^ (i >> 1);
                if (Ec < best || (Ec == best && rc < bestRow)) {
                    const int32_t d = Ec - best;
                    best = Ec;
                    bestRow = rc;
                    itemE = Ec;
                    itemRow = rc;
                    found = 1;
                    if constexpr (TIER == 1) {
                        static_for<0, kPatterns>([&](auto pc) { THR[decltype(pc)::value] += d; });
                    } else {
                        static_for<0, SEG>([&](auto pc) { TP[decltype(pc)::value] += d; });
                    }
                }
            }
        };

        // TIER 3 candidate: the chunk key (E_p + chunk minimum, row) enters
        // the wave's list if the list has room or the key beats its largest;
        // the threshold is then min(largest key's E when full, shared bound).
        auto candidate3 = [&](int32_t lm, int32_t thr, uint64_t i) {
            if (__builtin_amdgcn_ballot_w64(lm <= thr)) {
                const int32_t Ec = wave_min(lm) + (best - thr);
                if (Ec <= best) {
                    const int32_t nb = sread(tk_insert(Ec, i ^ (i >> 1)));
                    const int32_t d = nb - best;
                    best = nb;
                    static_for<0, SEG>([&](auto pc) { TP[decltype(pc)::value] += d; });
                }
            }
        };

        // Low flip of static level t (< kLowLevels) with static direction (Alg. 2:
        // E_sd += delta M_int[k]).
        auto low_flip = [&](auto tc, auto upc) {
            constexpr int t = decltype(tc)::value;
            constexpr bool up = decltype(upc)::value;
            if constexpr (LR && (t == 3 || t == 4)) {
#pragma unroll
                for (int j = 0; j < MC; j++) {
                    const int32_t r = ldsR[(t - 3) * (MC * kWave) + j * kWave + lane];
                    E[j] = up ? E[j] + r : E[j] - r;
                }
            } else {
#pragma unroll
                for (int j = 0; j < MC; j++) E[j] = up ? E[j] + R[t][j] : E[j] - R[t][j];
            }
            pin_vec<MC>(E);
        };
        // Flip of level kLowLevels in the middle of super-block sb (its
        // direction alternates between super-blocks).
        auto middle_flip = [&](uint64_t sb) {
            const bool up = (sb & 1) == 0;
            constexpr int tm = kLowLevels;
            if constexpr (G > tm) {
                if (up) {
#pragma unroll
                    for (int j = 0; j < MC; j++) E[j] += R[tm][j];
                } else {
#pragma unroll
                    for (int j = 0; j < MC; j++) E[j] -= R[tm][j];
                }
            } else {
                const int ws = up ? A - 1 - tm : 2 * A - 1 - tm;
#pragma unroll
                for (int j = 0; j < MC; j++) E[j] += trow(M, ws)[j * kWave + ulane];
            }
            pin_vec<MC>(E);
            nonlow_flip(A - 1 - tm, up, up ? Smid : -Smid, SmidL);
            return up;
        };
        // Flip entering super-block sb + 1 (Gray level >= kSuperLog).
        auto boundary_flip = [&](uint64_t sb) {
            const uint64_t ip1 = (sb + 1) << kSuperLog;
            const int t = __builtin_ctzll(ip1);
            const bool up = ((ip1 >> (t + 1)) & 1) == 0;
            const int w = A - 1 - t;
            bool done = false;
            static_for<kSuperLog, G>([&](auto tc) {
                constexpr int tt = decltype(tc)::value;
                if (t == tt) {
                    if (up) {
#pragma unroll
                        for (int j = 0; j < MC; j++) E[j] += R[tt][j];
                    } else {
#pragma unroll
                        for (int j = 0; j < MC; j++) E[j] -= R[tt][j];
                    }
                    done = true;
                }
            });
            // signed row (M_int or its negation) for levels read from L2:
            // one code path whatever the direction
            const int ws = up ? w : w + A;
            if (!done) {
#pragma unroll
                for (int j = 0; j < MC; j++) E[j] += trow(M, ws)[j * kWave + ulane];
            }
            pin_vec<MC>(E);
            int32_t SLw[kLowLevels];
            static_for<0, kLowLevels>([&](auto tc) {
                constexpr int tt = decltype(tc)::value;
                SLw[tt] = kall[kbase + kKBound + w * kLowLevels + tt];
            });
            nonlow_flip(w, up, S[size_t(ws) * kWave + ulane], SLw);
        };

        if constexpr (TIER == 1) {
            for (uint64_t sb = sb0; sb < sbEnd; sb++) {
                static_for<0, (1 << kSuperLog)>([&](auto oc) {
                    constexpr int o = decltype(oc)::value;
                    constexpr int pat = (o ^ (o >> 1)) & (kPatterns - 1);
                    candidate(tree_min<MC>(E), THR[pat], (sb << kSuperLog) | uint64_t(o));
                    if constexpr (o < (1 << kSuperLog) - 1) {
                        constexpr int t = cx_ctz(o + 1);
                        if constexpr (t < kLowLevels) {
                            constexpr bool up = ((((o + 1) ^ ((o + 1) >> 1)) >> t) & 1) != 0;
                            low_flip(std::integral_constant<int, t>{}, std::integral_constant<bool, up>{});
                        } else {
                            middle_flip(sb);
                            build_thr();
                        }
                    } else if (sb + 1 < sbEnd) {
                        boundary_flip(sb);
                        build_thr();
                    }
                });
            }
        } else {
            // 32-bit trip count: a 64-bit compare would take the vector unit
            const uint32_t nsb = uint32_t(sbEnd - sb0);
            for (uint32_t ks = 0; ks < nsb; ks++) {
                const uint64_t sb = sb0 + ks;
                lm0 = tree_min<MC>(E);
                tab2 = 0;
                // four 16-step segments, each with (cold) or without the
                // per-step bound tests; every step's chunk energies stay
                // observable through the (rarely taken) test, so each state
                // gets its add
                static_for<0, kSegs>([&](auto sc) {
                    constexpr int h = decltype(sc)::value;
                    // exact test of step o (cold path)
                    auto step_check = [&](auto oc) {
                        constexpr int o2 = decltype(oc)::value;
                        constexpr int o = h * SEG + o2;
                        if (W0 <= TP[o2]) {
                            const int32_t thr =
                                TP[o2] + kall[kbase + (3 + tab2) * kPatterns + (o & (kPatterns - 1))];
                            if constexpr (TIER == 3)
                                candidate3(tree_min<MC>(E), thr, (sb << kSuperLog) | uint64_t(o));
                            else
                                candidate(tree_min<MC>(E), thr, (sb << kSuperLog) | uint64_t(o));
                        }
                    };
                    // the low flip after step o (none after the segment's last)
                    auto step_flip = [&](auto oc) {
                        constexpr int o2 = decltype(oc)::value;
                        constexpr int o = h * SEG + o2;
                        if constexpr (o2 < SEG - 1) {
                            constexpr int t = cx_ctz(o + 1);
                            constexpr bool up = ((((o + 1) ^ ((o + 1) >> 1)) >> t) & 1) != 0;
                            low_flip(std::integral_constant<int, t>{},
                                     std::integral_constant<bool, up>{});
                        }
                    };
                    // One scalar test for the segment: an upper bound of its 16
                    // thresholds tp(o) = best - Enl - hs(o) - C2(o), since
                    // hs(o) >= sum_t min(0, H[t]) and C2(o) >= the segment's
                    // minimum of C2; any lane at or below it takes the cold
                    // path (the wave minimum W0 is formed only then)
                    int32_t tb = best - Enl - kall[kbase + kKC2Min + tab2 * 2 + (h & 1)];
                    static_for<0, kLowLevels>([&](auto tc) { tb -= min(0, H[decltype(tc)::value]); });
                    const bool cold = __builtin_amdgcn_ballot_w64(lm0 <= tb) != 0;
                    if (__builtin_expect(cold, 0)) {
                        W0 = wave_min_bcast(lm0);
                        build_tp(sc, tab2);
                        static_for<0, SEG>([&](auto oc) {
                            step_check(oc);
                            step_flip(oc);
                        });
                    } else {
                        static_for<0, SEG>([&](auto oc) { step_flip(oc); });
                    }
                    // the flip after the segment's last step: level 5 in the
                    // middle, level 4 (static direction) after segments 0 and
                    // 2, the boundary flip after the last
                    if constexpr (h == kSegs / 2 - 1) {
                        tab2 = middle_flip(sb) ? 1 : 2;
                    } else if constexpr (h < kSegs - 1) {
                        constexpr int o = (h + 1) * SEG;
                        constexpr int t = cx_ctz(o);
                        constexpr bool up = (((o ^ (o >> 1)) >> t) & 1) != 0;
                        low_flip(std::integral_constant<int, t>{}, std::integral_constant<bool, up>{});
                    } else if (ks + 1 < nsb) {
                        boundary_flip(sb);
                    }
                });
            }
        }

        if (TIER != 3 && found && lane == 0) {
            // Only items that found a candidate leave a record, marked in the
            // instance's bitmap (the record and bitmap pointers are read from
            // the descriptor here, on this rare path, rather than held in
            // registers through the walk).
            ItemRes r;
            r.E = itemE;
            r.found = 1;
            r.row = itemRow;
            const uint64_t q = g - item_begin;
            insts[cur].res[q] = r;
            const uint64_t b = insts[cur].bit0 + q;
            atomicOr(insts[cur].bits + (b >> 5), 1u << (b & 31));
            // publish once per item: every wave starting an item of this
            // instance at once would otherwise contend on one address
            atomicMin(gbest, itemE);
        }
    }
    if constexpr (TIER == 3) tk_flush();
}

// ---------------------------------------------------------------- finish

// Lexicographic (E, index) minimum over the block: butterflies inside each
// wave, then the wave results through LDS (sE, sI: one slot per wave).
__device__ void block_lexmin(int64_t &bE, uint64_t &bI, int64_t *sE, uint64_t *sI)
{
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        const int64_t e = __shfl_xor(bE, off, kWave);
        const uint64_t i = __shfl_xor(bI, off, kWave);
        lexmin(bE, bI, e, i);
    }
    const int w = int(threadIdx.x) / kWave, nw = int(blockDim.x) / kWave;
    if (int(threadIdx.x) % kWave == 0) {
        sE[w] = bE;
        sI[w] = bI;
    }
    __syncthreads();
    bE = INT64_MAX;
    bI = ~0ull;
    for (int k = 0; k < nw; k++) lexmin(bE, bI, sE[k], sI[k]);
    __syncthreads();
}

// Energy of U_N row idx from T staged in LDS, one lane per variable (the
// whole wave must call it): the same sum as energy_int.
__device__ int64_t wave_energy(const int32_t *T, int n, uint64_t idx)
{
    const int l = int(threadIdx.x) % kWave;
    int64_t part = 0;
    if (l < n && ((idx >> (n - 1 - l)) & 1)) {
        for (int j = l; j < n; j++)
            if ((idx >> (n - 1 - j)) & 1) part += T[l * n + j];
    }
    return wave_sum64(part);
}

constexpr int kFinishThreads = 1024;

__global__ __launch_bounds__(kFinishThreads) void finish_kernel(const Inst *__restrict__ insts,
                                                                FinalRes *__restrict__ out)
{
    __shared__ int64_t sE[kFinishThreads / kWave];
    __shared__ uint64_t sI[kFinishThreads / kWave];
    __shared__ int64_t sC[kMaxVars];   // suffix fields of the winning chunk
    __shared__ int64_t sEp;            // its prefix energy
    // T (and the caller's float32 Q) staged in LDS: every energy below reads
    // entries of T, and the float64 rescore runs on one thread in a fixed
    // order, where global-memory latency would dominate
    __shared__ int32_t sT[kMaxVars * kMaxVars];
    __shared__ float sQ[kMaxVars * kMaxVars];
    const Inst I = insts[blockIdx.x];
    const int n = I.n;
    for (int e = int(threadIdx.x); e < n * n; e += int(blockDim.x)) {
        sT[e] = I.T[e];
        if (I.Qf) sQ[e] = I.Qf[e];
    }
    __syncthreads();
    int64_t bE = INT64_MAX;
    uint64_t bI = ~0ull;
    int32_t status = 0;
    if (I.direct) {
        const uint64_t N = 1ull << n;
        for (uint64_t r = threadIdx.x; r < N; r += blockDim.x) lexmin(bE, bI, energy_int(sT, n, r), r);
        block_lexmin(bE, bI, sE, sI);
    } else {
        // the records of items whose bit is set (the others were never written)
        const uint64_t words = (I.n_items + 31) / 32;
        for (uint64_t w = threadIdx.x; w < words; w += blockDim.x) {
            uint32_t x = I.bits[w];
            while (x) {
                const uint32_t b = uint32_t(__builtin_ctz(x));
                x &= x - 1u;
                const ItemRes r = I.res[w * 32 + b];
                lexmin(bE, bI, r.E, r.row);
            }
        }
        block_lexmin(bE, bI, sE, sI);
        const int64_t Estar = bE;
        const uint64_t rowstar = bI;
        if (Estar == INT64_MAX) {
            status = 2;   // no item reported a candidate
        } else {
            // Argmin reconstruction (ConstructState of Alg. 2): the lowest
            // suffix s of chunk rowstar whose energy equals E*, from T.  With
            // the prefix fixed, E(row, s) = E_p(row) + sum_{t in s} c_t +
            // sum_{t < u in s} T[A+t][A+u] (Sec. II-C), where c_t = T[A+t][A+t]
            // + sum over the set prefix variables v of T[v][A+t].
            const int A = I.A, B = I.B;
            if (threadIdx.x < kWave) {
                const int l = int(threadIdx.x);
                int64_t part = 0;
                if (l < A && ((rowstar >> (A - 1 - l)) & 1)) {
                    for (int j = l; j < A; j++)
                        if ((rowstar >> (A - 1 - j)) & 1) part += sT[l * n + j];
                }
                part = wave_sum64(part);
                if (l == 0) sEp = part;
                if (l < B) {
                    int64_t c = sT[(A + l) * n + (A + l)];
                    for (int v = 0; v < A; v++)
                        if ((rowstar >> (A - 1 - v)) & 1) c += sT[v * n + A + l];
                    sC[l] = c;
                }
            }
            __syncthreads();
            bE = INT64_MAX;
            bI = ~0ull;
            const uint32_t NS = 1u << B;
            for (uint32_t s = threadIdx.x; s < NS; s += blockDim.x) {
                int64_t e = sEp;
                for (int t = 0; t < B; t++) {
                    if (!((s >> (B - 1 - t)) & 1)) continue;
                    e += sC[t];
                    for (int u = t + 1; u < B; u++)
                        if ((s >> (B - 1 - u)) & 1) e += sT[(A + t) * n + A + u];
                }
                if (e == Estar) lexmin(bE, bI, e, (rowstar << B) | s);
            }
            block_lexmin(bE, bI, sE, sI);
            if (bE != Estar) {
                status = 3;   // the walk claimed an energy the chunk lacks
            } else if (threadIdx.x < kWave) {
                // the winner evaluated in full from T must agree
                if (wave_energy(sT, n, bI) != Estar) status = 3;
            }
        }
    }
    if (threadIdx.x == 0) {
        FinalRes o;
        o.E = bE;
        o.index = bI;
        o.E64 = (I.Qf && status == 0) ? energy_f64(sQ, n, bI) : double(bE);
        o.status = status;
        o.pad = 0;
        out[blockIdx.x] = o;
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_tables(const Inst *d_insts, int n_inst, int max_A, unsigned long long *d_counters,
                         int n_counters, hipStream_t stream)
{
    // a few blocks per instance: each builds the partial sums it needs, so
    // more blocks mostly add scheduling work (4096-instance batches)
    int bx = (max_A * 1024 + 4095) / 4096;
    if (bx < 1) bx = 1;
    if (bx > 8) bx = 8;
    hipLaunchKernelGGL(tables_kernel, dim3(bx, n_inst), dim3(256), 0, stream, d_insts, d_counters,
                       n_counters);
    return hipGetLastError();
}

template <int MC, int G, bool LR = false>
static size_t walk_lds_bytes(int tier, int k)
{
    return lds_rows_offset(tier, k) + (LR ? lds_rows_bytes<MC>() : 0);
}

template <int MC, int G, bool LR = false>
static hipError_t launch_walk_g(int tier, const Inst *d_insts, int n_inst, uint64_t total_items,
                                unsigned long long *d_counter, const int32_t *d_k, int waves,
                                hipStream_t stream, const TopkWalk *tk)
{
    TopkWalk none{};
    if (tier == 1) {
        hipLaunchKernelGGL((walk_kernel<MC, G, 1, LR>), dim3(waves), dim3(kWave),
                           (walk_lds_bytes<MC, G, LR>(1, 0)), stream, d_insts, n_inst, total_items,
                           d_counter, d_k, none);
    } else if (tier == 2) {
        hipLaunchKernelGGL((walk_kernel<MC, G, 2, LR>), dim3(waves), dim3(kWave),
                           (walk_lds_bytes<MC, G, LR>(2, 0)), stream, d_insts, n_inst, total_items,
                           d_counter, d_k, none);
    } else if (tier == 3) {
        if (!tk || tk->k < 2 || n_inst != 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL((walk_kernel<MC, G, 3, LR>), dim3(waves), dim3(kWave),
                           (walk_lds_bytes<MC, G, LR>(3, tk->k)), stream, d_insts, n_inst,
                           total_items, d_counter, d_k, *tk);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MC, int G, bool LR = false>
static int occupancy_g(int tier, int topk_k)
{
    int blocks = 0;
    hipError_t e;
    if (tier == 3)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_kernel<MC, G, 3, LR>, kWave,
                                                         walk_lds_bytes<MC, G, LR>(3, topk_k));
    else if (tier == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_kernel<MC, G, 2, LR>, kWave,
                                                         walk_lds_bytes<MC, G, LR>(2, 0));
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_kernel<MC, G, 1, LR>, kWave,
                                                         walk_lds_bytes<MC, G, LR>(1, 0));
    if (e != hipSuccess || blocks < 1) return 1;
    return blocks;
}

// Variants built: every MC with G = 12; MC = 8 and 16 with G = 8; MC = 16
// with G = 6 and 5, "4": G = 6 with levels 3 and 4 in LDS (levels 0-2 and 5
// in VGPRs, four waves per SIMD), and "3": G = 5 with levels 3 and 4 in LDS
// (levels 0-2 in VGPRs; every flip of level 5 or above reads its signed row
// from L2, so the flip into the next super-block takes one code path).
bool walk_variant_exists(int mcols, int vgpr_levels)
{
    if (vgpr_levels == 12) return mcols == 1 || mcols == 2 || mcols == 4 || mcols == 8 || mcols == 16;
    if (vgpr_levels == 8) return mcols == 8 || mcols == 16;
    if (vgpr_levels == 6 || vgpr_levels == 5 || vgpr_levels == 4 || vgpr_levels == 3)
        return mcols == 16;
    return false;
}

int walk_occupancy(int mcols, int vgpr_levels, int tier, int topk_k)
{
    if (vgpr_levels == 4) return occupancy_g<16, 6, true>(tier, topk_k);
    if (vgpr_levels == 3) return occupancy_g<16, 5, true>(tier, topk_k);
    if (vgpr_levels == 5) return occupancy_g<16, 5>(tier, topk_k);
    if (vgpr_levels == 6) return occupancy_g<16, 6>(tier, topk_k);
    if (vgpr_levels == 8)
        return mcols == 8 ? occupancy_g<8, 8>(tier, topk_k) : occupancy_g<16, 8>(tier, topk_k);
    switch (mcols) {
    case 1: return occupancy_g<1, 12>(tier, topk_k);
    case 2: return occupancy_g<2, 12>(tier, topk_k);
    case 4: return occupancy_g<4, 12>(tier, topk_k);
    case 8: return occupancy_g<8, 12>(tier, topk_k);
    default: return occupancy_g<16, 12>(tier, topk_k);
    }
}

hipError_t launch_walk(int mcols, int vgpr_levels, int tier, const Inst *d_insts, int n_inst,
                       uint64_t total_items, unsigned long long *d_counter, const int32_t *d_k,
                       int waves, hipStream_t stream, const TopkWalk *tk)
{
#define QK_ARGS tier, d_insts, n_inst, total_items, d_counter, d_k, waves, stream, tk
    if (vgpr_levels == 6 || vgpr_levels == 5 || vgpr_levels == 4 || vgpr_levels == 3) {
        if (mcols != 16) return hipErrorInvalidValue;
        if (vgpr_levels == 4) return launch_walk_g<16, 6, true>(QK_ARGS);
        if (vgpr_levels == 3) return launch_walk_g<16, 5, true>(QK_ARGS);
        return vgpr_levels == 6 ? launch_walk_g<16, 6>(QK_ARGS) : launch_walk_g<16, 5>(QK_ARGS);
    }
    if (vgpr_levels == 8) {
        if (mcols == 8) return launch_walk_g<8, 8>(QK_ARGS);
        if (mcols == 16) return launch_walk_g<16, 8>(QK_ARGS);
        return hipErrorInvalidValue;
    }
    if (vgpr_levels != 12) return hipErrorInvalidValue;
    switch (mcols) {
    case 1: return launch_walk_g<1, 12>(QK_ARGS);
    case 2: return launch_walk_g<2, 12>(QK_ARGS);
    case 4: return launch_walk_g<4, 12>(QK_ARGS);
    case 8: return launch_walk_g<8, 12>(QK_ARGS);
    case 16: return launch_walk_g<16, 12>(QK_ARGS);
    default: return hipErrorInvalidValue;
    }
#undef QK_ARGS
}

hipError_t launch_finish(const Inst *d_insts, int n_inst, FinalRes *d_out, hipStream_t stream)
{
    hipLaunchKernelGGL(finish_kernel, dim3(n_inst), dim3(kFinishThreads), 0, stream, d_insts, d_out);
    return hipGetLastError();
}

}  // namespace qk

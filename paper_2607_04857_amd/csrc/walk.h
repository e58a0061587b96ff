// walk.h -- the Gray-walk kernel template (Sec. III-B, Eq. incremental_update)
// and its per-variant launch helpers.  Each walk_*.hip file instantiates a
// few variants, so that the variants compile in parallel.
#pragma once

#include "kcommon.h"
#include "walk_variants.h"

namespace qk {

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
//         only the scalar test W0 <= THR - D(o).  Each 32-step segment (a
//         half super-block: the level-5 flip separates the two) first tests
//         lm0 against an upper bound of its 32 thresholds (one vector
//         compare); only when a lane passes are W0 and the exact thresholds
//         formed and tested, step by step.
// TIER 4, 5: tiers 2 and 3 on the packed layout: each of the MC words of a
//         lane holds two chunk energies (columns c and c + 2^(B-1) of the
//         chunk), so one 32-bit add per word and step moves two states (Eq.
//         incremental_update at 16-bit precision); only the lane minimum
//         (packed 16-bit minima, then the unbiased smaller half) and the
//         prefix energy's shift differ.
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

// Bytes of dynamic LDS ahead of the LDS rows (the tier-3 / tier-5 list),
// 16-aligned.
__host__ __device__ inline size_t lds_rows_offset(int tier, int k)
{
    (void)k;
    return (tier == 3 || tier == 5) ? (topk_lds_bytes() + 15) & ~size_t(15) : 0;
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
        M[5] = tk.prep ? tk.prep->hist_shift : tk.hist_shift;
        P[0] = 0;
        P[1] = reinterpret_cast<uint64_t>(tk.gthr);
        P[2] = reinterpret_cast<uint64_t>(tk.listE);
        P[3] = reinterpret_cast<uint64_t>(tk.listR);
        P[4] = reinterpret_cast<uint64_t>(tk.listCount);
        P[5] = reinterpret_cast<uint64_t>(tk.hist);
        P[6] = reinterpret_cast<uint64_t>(tk.lowbin);
        P[7] = uint64_t(tk.prep ? tk.prep->hist_lo : tk.hist_lo);
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
    static_assert(TIER >= 1 && TIER <= 5, "tier");
    static_assert(G >= kLowLevels && G <= kMaxVgprLevels, "VGPR-resident levels");
    // packed layout (tiers 4 and 5) and the test it runs (2: best, 3: top-k)
    constexpr bool PK = TIER >= 4;
    constexpr int BT = PK ? TIER - 2 : TIER;
    // steps per bound-test segment: tier 3's looser threshold takes the
    // exact path more often, where shorter segments and SGPR thresholds pay
    constexpr int SEG = BT == 3 ? kSegStepsTopk : kSegSteps;
    constexpr int NSEG = (1 << kSuperLog) / SEG;
    const int lane = int(threadIdx.x);
    const uint32_t ulane = threadIdx.x;
    // row v of a lane-major [rows][MC*64] table: uniform base pointer
    auto trow = [](const gint32 *t, int v) { return t + size_t(v) * (MC * kWave); };
    // this lane's chunk minimum (packed: over both halves of every word)
    auto lane_min = [](const int32_t(&e)[MC]) {
        if constexpr (PK) return tree_min_packed<MC>(e);
        else return tree_min<MC>(e);
    };
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

    if constexpr (BT == 3) tk_init(tk);

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
            if constexpr (BT != 3) gbest = I.gbest;
        }

        // Best energy found by any wave for this instance (published at the
        // end of each item): a chunk can improve the final answer only if its
        // key is at most that.  (A chunk tying it with an unknown row is still
        // recorded: bestRow restarts at the largest row whenever the shared
        // value lowers best.)
        if constexpr (BT != 3) {
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
        // F: field of every prefix variable from the non-low ones (levels >=
        // kLowLevels, variables 0..A-1-kLowLevels), plus its diagonal; one
        // lane per variable.
        const int32_t diagl = lane < A ? Tm[lane * nT + lane] : 0;   // T[l][l], lane l < A
        int32_t F = diagl;
        for (int w = 0; w <= A - 1 - kLowLevels; w++)
            if ((row0 >> (A - 1 - w)) & 1) F += S[size_t(w) * kWave + ulane];
        // E_nl = energy of the non-low prefix bits = (sum_set F_w + T_ww) / 2
        const bool lbit = lane <= A - 1 - kLowLevels && ((row0 >> (A - 1 - lane)) & 1);
        int32_t Enl = int32_t(wave_sum64(lbit ? int64_t(F) + diagl : 0) / 2);
        // the chunk energies carry the instance's shift c (packed: into the
        // 16-bit range; int32: non-negative), the prefix energy the opposite
        // one, so every sum is the true energy
        Enl -= insts[cur].pack_shift;
        Enl = sread(Enl);
        int32_t H[kLowLevels];
        static_for<0, kLowLevels>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            H[t] = __builtin_amdgcn_readlane(F, A - 1 - t);
        });
        if constexpr (BT == 3) best = tk_threshold();

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
        // TIER 3: for the SEG offsets o of segment `seg` (o = SEG seg + o2),
        //   tp(o) = best - E_p(low pattern at o) - C2(o)   (K table tab),
        // computed by walking the Gray sequence of patterns g(o) & 31 from
        // the segment's first one; hs = the sum of H[t] over the set low
        // bits.  f(o2, tp) is called for every offset.  Step o can hold a
        // candidate only if W0 <= tp(o).
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
        // Tier-3 thresholds of the current segment, kept in SGPRs.
        int32_t TP[BT == 3 ? SEG : 1];
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
                    if constexpr (BT == 3)
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
                lm0 = lane_min(E);
                tab2 = 0;
                // NSEG segments of SEG steps (tier 2: the two halves around
                // the level-5 flip), each with (cold) or without the per-step
                // bound tests; every step's chunk energies stay observable
                // through the (rarely taken) test, so each state gets its add
                static_for<0, NSEG>([&](auto sc) {
                    constexpr int h = decltype(sc)::value;
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
                    // One scalar test for the segment: an upper bound of its SEG
                    // thresholds tp(o) = best - Enl - hs(o) - C2(o), since
                    // hs(o) >= sum_t min(0, H[t]) and C2(o) >= the segment's
                    // minimum of C2; any lane at or below it takes the cold
                    // path (the wave minimum W0 is formed only then)
                    int32_t tb = best - Enl - kall[kbase + kc2min_slot(SEG, tab2, h)];
                    static_for<0, kLowLevels>([&](auto tc) { tb -= min(0, H[decltype(tc)::value]); });
                    const bool cold = __builtin_amdgcn_ballot_w64(lm0 <= tb) != 0;
                    if constexpr (BT == 3) {
                        if (__builtin_expect(cold, 0)) {
                            // exact tests against the segment's SGPR thresholds
                            W0 = wave_min_bcast(lm0);
                            build_tp(sc, tab2);
                            static_for<0, SEG>([&](auto oc) {
                                constexpr int o2 = decltype(oc)::value;
                                constexpr int o = h * SEG + o2;
                                if (W0 <= TP[o2]) {
                                    const int32_t thr =
                                        TP[o2] + kall[kbase + (3 + tab2) * kPatterns + (o & (kPatterns - 1))];
                                    candidate3(lane_min(E), thr, (sb << kSuperLog) | uint64_t(o));
                                }
                                step_flip(oc);
                            });
                        } else {
                            static_for<0, SEG>([&](auto oc) { step_flip(oc); });
                        }
                    } else {
                        if (__builtin_expect(cold, 0)) {
                            // Exact tests, step by step: at offset o,
                            //   tp(o) = best - E_p(low pattern at o) - C2(o)
                            // (K table tab2), with hs = the sum of H[t] over the
                            // set low bits walked along the Gray sequence of
                            // patterns g(o) & 31 and best read afresh at every
                            // step (a candidate found earlier in the segment has
                            // lowered it).  Step o can hold a candidate only if
                            // W0 <= tp(o), and then holds one exactly when the
                            // chunk minimum is <= tp(o) + D(o) = best - E_p(o).
                            W0 = wave_min_bcast(lm0);
                            constexpr int o0 = h * SEG;
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
                                const int32_t tp = (best - Enl) - hs -
                                                   kall[kbase + tab2 * kPatterns + (o & (kPatterns - 1))];
                                if (W0 <= tp) {
                                    const int32_t thr =
                                        tp + kall[kbase + (3 + tab2) * kPatterns + (o & (kPatterns - 1))];
                                    candidate(lane_min(E), thr, (sb << kSuperLog) | uint64_t(o));
                                }
                                step_flip(oc);
                            });
                        } else {
                            static_for<0, SEG>([&](auto oc) { step_flip(oc); });
                        }
                    }
                    // the flip after the segment's last step: level 5 in the
                    // middle, a low level (static direction) between shorter
                    // segments, the boundary flip after the last
                    if constexpr (h == NSEG / 2 - 1) {
                        tab2 = middle_flip(sb) ? 1 : 2;
                    } else if constexpr (h < NSEG - 1) {
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

        if (BT != 3 && found && lane == 0) {
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
    if constexpr (BT == 3) tk_flush();
}

template <int MC, int G, bool LR = false>
static size_t walk_lds_bytes(int tier, int k)
{
    return lds_rows_offset(tier, k) + (LR ? lds_rows_bytes<MC>() : 0);
}

template <int MC, int G, bool LR = false>
static hipError_t launch_walk_g(const WalkLaunch &w)
{
    TopkWalk none{};
    if (w.tier == 1) {
        hipLaunchKernelGGL((walk_kernel<MC, G, 1, LR>), dim3(w.waves), dim3(kWave),
                           (walk_lds_bytes<MC, G, LR>(1, 0)), w.stream, w.insts, w.n_inst,
                           w.total_items, w.counter, w.k, none);
    } else if (w.tier == 2) {
        hipLaunchKernelGGL((walk_kernel<MC, G, 2, LR>), dim3(w.waves), dim3(kWave),
                           (walk_lds_bytes<MC, G, LR>(2, 0)), w.stream, w.insts, w.n_inst,
                           w.total_items, w.counter, w.k, none);
    } else if (w.tier == 4 && MC >= 4) {
        if constexpr (MC >= 4)
            hipLaunchKernelGGL((walk_kernel<MC, G, 4, LR>), dim3(w.waves), dim3(kWave),
                               (walk_lds_bytes<MC, G, LR>(4, 0)), w.stream, w.insts, w.n_inst,
                               w.total_items, w.counter, w.k, none);
    } else if (w.tier == 3) {
        if (!w.tk || w.tk->k < 2 || w.n_inst != 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL((walk_kernel<MC, G, 3, LR>), dim3(w.waves), dim3(kWave),
                           (walk_lds_bytes<MC, G, LR>(3, w.tk->k)), w.stream, w.insts, w.n_inst,
                           w.total_items, w.counter, w.k, *w.tk);
    } else if (w.tier == 5 && MC >= 4) {
        if (!w.tk || w.tk->k < 2 || w.n_inst != 1) return hipErrorInvalidValue;
        if constexpr (MC >= 4)
            hipLaunchKernelGGL((walk_kernel<MC, G, 5, LR>), dim3(w.waves), dim3(kWave),
                               (walk_lds_bytes<MC, G, LR>(5, w.tk->k)), w.stream, w.insts,
                               w.n_inst, w.total_items, w.counter, w.k, *w.tk);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MC, int G, bool LR = false>
static int occupancy_g(int tier, int topk_k)
{
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
    if (tier == 3)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_kernel<MC, G, 3, LR>, kWave,
                                                         walk_lds_bytes<MC, G, LR>(3, topk_k));
    else if (tier == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_kernel<MC, G, 2, LR>, kWave,
                                                         walk_lds_bytes<MC, G, LR>(2, 0));
    else if (tier == 4 && MC >= 4) {
        if constexpr (MC >= 4)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_kernel<MC, G, 4, LR>, kWave,
                                                             walk_lds_bytes<MC, G, LR>(4, 0));
    } else if (tier == 5 && MC >= 4) {
        if constexpr (MC >= 4)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_kernel<MC, G, 5, LR>, kWave,
                                                             walk_lds_bytes<MC, G, LR>(5, topk_k));
    }
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, walk_kernel<MC, G, 1, LR>, kWave,
                                                         walk_lds_bytes<MC, G, LR>(1, 0));
    if (e != hipSuccess || blocks < 1) return 1;
    return blocks;
}

}  // namespace qk

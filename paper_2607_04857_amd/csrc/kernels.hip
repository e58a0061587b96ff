// kernels.hip -- gfx950 kernels of the exhaustive dense-QUBO solver: the
// table build, the finish and the walk dispatch (the walk kernel itself is in
// walk.h, its variants in walk_*.hip).
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
//    once per 32 steps; exact per-step tests run only when that passes (tier
//    1 does the exact v_min3 test at every step).  Each step still updates
//    the chunk vector once (pinned, so the compiler cannot fold flips).  Ties
//    resolve to the lowest prefix row here and to the lowest suffix in the
//    final rescan, giving the lowest U_N index overall.
#include "kcommon.h"
#include "walk_variants.h"

namespace qk {

// ---------------------------------------------------------------- tables

// Greedy single-flip descents from two starts per wave (the all-zero state
// for wave 0's first start, hashed states otherwise), lowering the
// instance's shared best to the energy of the local minima found.  Any
// state's energy is a valid threshold for the walk (the state's own chunk
// still passes it), and a local minimum of a dense QUBO is usually close to
// the global one, so walk waves start with a near-final threshold.
__device__ void seed_best(const Inst &I, int wave)
{
    int32_t bestE = kNoEnergy;
    for (int rep = 0; rep < 2; rep++) {
        int32_t E;
        uint64_t xm;
        greedy_descent(I.T, I.n, uint32_t(wave) * 2u + uint32_t(rep), E, xm);
        bestE = min(bestE, E);
    }
    if (int(threadIdx.x) % kWave == 0) atomicMin(I.gbest, bestE);
}

__global__ __launch_bounds__(256) void tables_kernel(const Inst *__restrict__ insts,
                                                     unsigned long long *__restrict__ counters,
                                                     int n_counters)
{
    const Inst I = insts[blockIdx.y];
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        // a device-prepared instance whose input was refused walks no item
        const unsigned long long c0 = (I.prep && I.prep->status != 0) ? (1ull << 62) : 0ull;
        for (int c = int(threadIdx.x); c < n_counters; c += int(blockDim.x)) counters[c] = c0;
    }
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
    // lowest bits of s and part[v][32 + (s >> 5)] over the others (B <= 11).
    constexpr int kPartW = 32 + 64;
    __shared__ int32_t part[kMaxPrefixRows][kPartW];
    const uint32_t pw = 32u + (NS >> 5);
    for (uint32_t e = threadIdx.x; e < uint32_t(A) * pw; e += blockDim.x) {
        const int v = int(e / pw), x = int(e % pw);
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
    auto mval = [&](int v, uint32_t s) { return part[v][s & 31u] + part[v][32u + (s >> 5)]; };
    // E_s(U_B)[s] = sum_{t <= u, both set} T[A+t][A+u] (Sec. III-A, step 2)
    auto esuf = [&](uint32_t s) {
        int32_t acc = 0;
        for (int t = 0; t < B; t++) {
            if (!((s >> (B - 1 - t)) & 1u)) continue;
            for (int u = t; u < B; u++)
                if ((s >> (B - 1 - u)) & 1u) acc += T[(A + t) * n + A + u];
        }
        return acc;
    };
    // rows A..2A-1 hold -M_int: a flip whose direction is known only at
    // run time then adds one row or the other, without a branch.  Packed:
    // word c of a row is m(c) + m(c + NW) 2^16 and its negation the
    // negated word (both mod 2^32, the packed map being additive).
    const int lw = I.packed ? B - 1 : B;
    const uint32_t NW = 1u << lw;   // words per row
    for (uint32_t e = tid; e < uint32_t(A) * NW; e += stride) {
        const int v = int(e >> lw);
        const uint32_t c = e & (NW - 1);
        uint32_t m = uint32_t(mval(v, c));
        if (I.packed) m += uint32_t(mval(v, c + NW)) << 16;
        I.M[e] = int32_t(m);
        I.M[uint32_t(A) * NW + e] = int32_t(0u - m);
    }
    for (uint32_t c = tid; c < NW; c += stride) {
        if (I.packed) {
            const int32_t b = I.pack_shift + kPackBias;
            I.EB[c] = int32_t(uint32_t(esuf(c) + b) + (uint32_t(esuf(c + NW) + b) << 16));
        }
        else
            I.EB[c] = esuf(c) + I.pack_shift;
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
    constexpr int kCols = 2048 / 256;  // columns per thread (B <= 11)
    int32_t mcol[kCols][kLowLevels + 1];   // M rows of levels 0..kLowLevels at this thread's columns
    for (int k = 0; k < kCols; k++) {
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
        for (int k = 0; k < kCols; k++) {
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
    if (threadIdx.x < 9) {   // min of C2 over each bound-test segment (kc2min_slot)
        const int x = int(threadIdx.x);
        const int tab = x < 3 ? x : (x - 3) / 2;
        const int lo = x < 3 ? 0 : ((x - 3) % 2) * 16, hi = x < 3 ? kPatterns : lo + 16;
        int32_t m = INT32_MAX;
        for (int oo = lo; oo < hi; oo++) m = min(m, c2s[tab * kPatterns + oo]);
        I.K[kKC2Min + x] = m;
    }
    if (threadIdx.x >= 9 && threadIdx.x < 12) I.K[kKC2Min + threadIdx.x] = 0;
}

// ---------------------------------------------------------------- prepare

// Canonicalisation of a lone instance held in device memory, with the host
// planner's arithmetic: fold T_ii = Q_ii, T_ij = Q_ij + Q_ji (i < j; the
// energy sums over all pairs); int32 input: sum |T| <= 2^30 - 1 proves every
// partial sum the walk forms exact in int32; float32 input: all entries
// finite, S = sum |T| in float64 accumulated i ascending then j ascending
// (the host's order, so the same S), p = the largest exponent with
// S 2^p <= 2^29, T~ = round-half-even(T 2^p).
constexpr int kPrepThreads = 1024;

__device__ __forceinline__ int prep_scale_exponent(double S)
{
    // S = m 2^e, m in [0.5, 1): m 2^(e+p) <= 2^29 for e + p <= 29, and for
    // e + p = 30 exactly when m = 0.5
    if (!(S > 0.0)) return 0;
    int e = 0;
    const double m = frexp(S, &e);
    return (m == 0.5 ? 30 : 29) - e;
}

__global__ __launch_bounds__(kPrepThreads) void prepare_kernel(const void *__restrict__ dQ, int n,
                                                               int is_fp32, int32_t *__restrict__ T,
                                                               PrepOut *__restrict__ out,
                                                               Inst *__restrict__ inst)
{
    __shared__ double sTd[kMaxVars * kMaxVars];   // folded float32 input in float64
    __shared__ int32_t sTi[kMaxVars * kMaxVars];  // the int32 T written to T
    __shared__ int32_t sPart[kMaxPrefixRows][64]; // M_int partial sums (see below)
    __shared__ long long sLo;
    __shared__ unsigned long long sSum;
    __shared__ int sNnz, sBad;
    __shared__ double sS;
    const int tid = int(threadIdx.x), nn = n * n;
    if (tid == 0) {
        sSum = 0ull;
        sNnz = 0;
        sBad = 0;
    }
    __syncthreads();
    uint64_t mySum = 0;
    int myNnz = 0, myBad = 0;
    if (!is_fp32) {
        const int32_t *q = static_cast<const int32_t *>(dQ);
        for (int e = tid; e < nn; e += kPrepThreads) {
            const int i = e / n, j = e % n;
            int32_t v = 0;
            if (i <= j) {
                const int64_t t = i == j ? int64_t(q[e]) : int64_t(q[e]) + int64_t(q[j * n + i]);
                mySum += uint64_t(t < 0 ? -t : t);
                v = int32_t(t);   // kept only if the bound holds (else T is zeroed)
            }
            T[e] = v;
            sTi[e] = v;
        }
    } else {
        const float *q = static_cast<const float *>(dQ);
        for (int e = tid; e < nn; e += kPrepThreads) {
            const int i = e / n, j = e % n;
            double t = 0.0;
            if (i <= j) {
                const double a = double(q[e]), b = i == j ? 0.0 : double(q[j * n + i]);
                if (!isfinite(a) || !isfinite(b)) myBad = 1;
                t = a + b;
                if (t != 0.0) myNnz++;
            }
            sTd[e] = t;
        }
    }
    atomicAdd(&sSum, (unsigned long long)mySum);
    atomicAdd(&sNnz, myNnz);
    atomicOr(&sBad, myBad);
    __syncthreads();
    int32_t status = 0;
    int p = 0;
    int64_t sum = 0;
    double eps = 0.0;
    if (!is_fp32) {
        sum = int64_t(sSum);
        if (sum > kExactSumLimit) status = kPrepOverflow;
    } else if (sBad) {
        status = kPrepNonFinite;
    } else {
        if (tid == 0) {
            double S = 0.0;
            for (int i = 0; i < n; i++)
                for (int j = i; j < n; j++) S += fabs(sTd[i * n + j]);
            sS = S;
            sSum = 0ull;
        }
        __syncthreads();
        p = prep_scale_exponent(sS);
        uint64_t s2 = 0;
        for (int e = tid; e < nn; e += kPrepThreads) {
            const int64_t t = int64_t(rint(ldexp(sTd[e], p)));   // ties to even
            s2 += uint64_t(t < 0 ? -t : t);
            T[e] = int32_t(t);
            sTi[e] = int32_t(t);
        }
        atomicAdd(&sSum, (unsigned long long)s2);
        __syncthreads();
        sum = int64_t(sSum);
        if (sum > kExactSumLimit) status = kPrepInternal;
        eps = double(sNnz) * ldexp(1.0, -p - 1);
    }
    if (status != 0)
        for (int e = tid; e < nn; e += kPrepThreads) T[e] = 0;
    // The int32 walk's shift c = -(least chunk energy of the split): every
    // E_sd(s, x_p) = E_s(s) + sum_v x_v M[v][s] is at least E_s(s) + the
    // negative M[v][s], so the least is the minimum of that over the 2^B
    // columns (the host planner's rule, with the same int32 bound).
    const int A = inst->A, B = inst->B;
    const bool walked = !inst->direct && status == 0;
    if (tid == 0) sLo = LLONG_MAX;
    __syncthreads();
    // M[v][s] as the table build forms it: the partial sums over the five
    // lowest bits of s and over the others (B <= 10 here: 32 + 32 entries)
    if (walked)
        for (int e = tid; e < A * 64; e += kPrepThreads) {
            const int v = e / 64, x = e % 64;
            int32_t acc = 0;
            if (x < 32) {
                for (int u = 0; u < 5 && u < B; u++)
                    if ((x >> u) & 1) acc += sTi[v * n + A + B - 1 - u];
            } else {
                for (int u = 0; u < B - 5; u++)
                    if (((x - 32) >> u) & 1) acc += sTi[v * n + A + B - 6 - u];
            }
            sPart[v][x] = acc;
        }
    __syncthreads();
    if (walked) {
        long long lo = LLONG_MAX;
        for (uint32_t c = uint32_t(tid); c < (1u << B); c += kPrepThreads) {
            int64_t e = 0;
            for (int t = 0; t < B; t++) {
                if (!((c >> (B - 1 - t)) & 1u)) continue;
                for (int u = t; u < B; u++)
                    if ((c >> (B - 1 - u)) & 1u) e += sTi[(A + t) * n + A + u];
            }
            for (int v = 0; v < A; v++) {
                const int32_t m = sPart[v][c & 31u] + sPart[v][32u + (c >> 5)];
                if (m < 0) e += m;
            }
            lo = e < lo ? e : lo;
        }
        atomicMin(&sLo, lo);
    }
    __syncthreads();
    if (tid == 0) {
        const int64_t lo = walked ? int64_t(sLo) : 0;
        inst->pack_shift = sum + (lo < 0 ? -lo : lo) <= kExactSumLimit ? int32_t(-lo) : 0;
    }
    if (tid == 0) {
        PrepOut o;
        o.status = status;
        o.p = status ? 0 : p;
        o.sum_abs = status ? 0 : sum;
        o.eps_q = status ? 0.0 : eps;
        int shift = 0;
        while (((2 * o.sum_abs) >> shift) >= kTopkBins) shift++;
        o.hist_lo = -o.sum_abs;
        o.hist_shift = shift;
        o.pad = 0;
        *out = o;
    }
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
        // the records of items whose bit is set (the others were never
        // written); each thread takes four consecutive bitmap words at a
        // time, loaded together before any is examined
        const uint64_t words = (I.n_items + 31) / 32;
        for (uint64_t w0 = uint64_t(threadIdx.x) * 4; w0 < words; w0 += uint64_t(blockDim.x) * 4) {
            uint32_t x[4];
#pragma unroll
            for (int k = 0; k < 4; k++) x[k] = w0 + k < words ? I.bits[w0 + k] : 0u;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                while (x[k]) {
                    const uint32_t b = uint32_t(__builtin_ctz(x[k]));
                    x[k] &= x[k] - 1u;
                    const ItemRes r = I.res[(w0 + k) * 32 + b];
                    lexmin(bE, bI, r.E, r.row);
                }
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
            const int w = int(threadIdx.x) / kWave, l = int(threadIdx.x) % kWave;
            auto set = [&](int v) { return ((rowstar >> (A - 1 - v)) & 1) != 0; };
            // E_p(row*): the pairs i <= j < A of set prefix variables, spread
            // over the block (a few per thread), one LDS add per wave
            if (threadIdx.x == 0) sEp = 0;
            __syncthreads();
            int64_t part = 0;
            for (int e = int(threadIdx.x); e < A * A; e += int(blockDim.x)) {
                const int i = e / A, j = e % A;
                if (j >= i && set(i) && set(j)) part += sT[i * n + j];
            }
            part = wave_sum64(part);
            if (l == 0 && part != 0) atomicAdd(reinterpret_cast<unsigned long long *>(&sEp),
                                               static_cast<unsigned long long>(part));
            // c_t: wave t sums the couplings of suffix variable A+t with the
            // set prefix variables, one lane per prefix variable (A < 64)
            if (w < B) {
                int64_t c = (l < A && set(l)) ? int64_t(sT[l * n + A + w]) : 0;
                c = wave_sum64(c);
                if (l == 0) sC[w] = c + sT[(A + w) * n + (A + w)];
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
            } else {
                // the winner evaluated in full from T must agree: its pairs
                // i <= j < n spread over the block as above
                if (threadIdx.x == 0) sEp = 0;
                __syncthreads();
                int64_t full = 0;
                for (int e = int(threadIdx.x); e < n * n; e += int(blockDim.x)) {
                    const int i = e / n, j = e % n;
                    if (j >= i && ((bI >> (n - 1 - i)) & 1) && ((bI >> (n - 1 - j)) & 1))
                        full += sT[i * n + j];
                }
                full = wave_sum64(full);
                if (l == 0 && full != 0) atomicAdd(reinterpret_cast<unsigned long long *>(&sEp),
                                                   static_cast<unsigned long long>(full));
                __syncthreads();
                if (sEp != Estar) status = 3;
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

hipError_t launch_prepare(const void *dQ, int n, int is_fp32, int32_t *d_T, PrepOut *d_prep,
                          Inst *d_inst, hipStream_t stream)
{
    if (n < 1 || n > kMaxVars) return hipErrorInvalidValue;
    hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(kPrepThreads), 0, stream, dQ, n, is_fp32, d_T,
                       d_prep, d_inst);
    return hipGetLastError();
}

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

// Variants built: every MC with G = 12; MC = 8 and 16 with G = 8; MC = 16
// with G = 6 and 5, "4": G = 6 with levels 3 and 4 in LDS (levels 0-2 and 5
// in VGPRs, four waves per SIMD), and "3": G = 5 with levels 3 and 4 in LDS
// (levels 0-2 in VGPRs; every flip of level 5 or above reads its signed row
// from L2).
bool walk_packed_exists(int mcols, int vgpr_levels)
{
    return mcols >= 4 && walk_variant_exists(mcols, vgpr_levels);
}

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
    switch (vgpr_levels) {
    case 4: return occupancy_walk_g6(true, tier, topk_k);
    case 3: return occupancy_walk_g5(true, tier, topk_k);
    case 6: return occupancy_walk_g6(false, tier, topk_k);
    case 5: return occupancy_walk_g5(false, tier, topk_k);
    case 8: return occupancy_walk_g8(mcols, tier, topk_k);
    default:
        return mcols <= 4 ? occupancy_walk_g12(mcols, tier, topk_k)
                          : occupancy_walk_g12w(mcols, tier, topk_k);
    }
}

hipError_t launch_walk(int mcols, int vgpr_levels, int tier, const Inst *d_insts, int n_inst,
                       uint64_t total_items, unsigned long long *d_counter, const int32_t *d_k,
                       int waves, hipStream_t stream, const TopkWalk *tk)
{
    const WalkLaunch w{tier, d_insts, n_inst, total_items, d_counter, d_k, waves, stream, tk};
    if (vgpr_levels == 6 || vgpr_levels == 5 || vgpr_levels == 4 || vgpr_levels == 3) {
        if (mcols != 16) return hipErrorInvalidValue;
        if (vgpr_levels == 6 || vgpr_levels == 4) return launch_walk_g6(vgpr_levels == 4, w);
        return launch_walk_g5(vgpr_levels == 3, w);
    }
    if (vgpr_levels == 8) return launch_walk_g8(mcols, w);
    if (vgpr_levels != 12) return hipErrorInvalidValue;
    return mcols <= 4 ? launch_walk_g12(mcols, w) : launch_walk_g12w(mcols, w);
}

hipError_t launch_finish(const Inst *d_insts, int n_inst, FinalRes *d_out, hipStream_t stream)
{
    hipLaunchKernelGGL(finish_kernel, dim3(n_inst), dim3(kFinishThreads), 0, stream, d_insts, d_out);
    return hipGetLastError();
}

}  // namespace qk

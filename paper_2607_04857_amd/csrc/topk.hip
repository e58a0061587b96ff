// topk.hip -- the k lowest-energy states of one instance (k > 1).
//
// The paper's kernel returns the minimum; it names the k lowest energies as
// an extension (Sec. VI).  Here the answer is the k smallest (E, index)
// pairs, index = U_N row.  Let a chunk be the 2^B states of one prefix row
// and its key (E_p + min over the chunk, row).  The k smallest states lie in
// the k smallest chunks by key: if a chunk c holding one of them were not
// among those, k chunks with smaller keys would each hold a state smaller
// than it.  So:
//   1. the tier-3 walk leaves per-wave lists of candidate chunk keys that
//      together contain the k smallest chunks (kernels.hip);
//   2. compact the list entries at or below the final shared bound, and
//      select the k smallest chunk keys among them;
//   3. rescan those chunks: every state's energy from the tables,
//      E = E_p(row) + E_s(s) + x_p M_int[:, s] (Sec. II-C), keeping the
//      states at or below the largest selected chunk key (the k chunk minima
//      are k states at or below it, so the k-th smallest energy is too);
//      an instance with fewer than k chunks keeps all of its states;
//   4. select the k smallest (E, index) among them, sorted;
//   5. verify each energy from T, rescore fp32 instances in float64 and sort
//      those by (E64, index).
// Selection is an exact radix select on the energy (order-preserving
// unsigned key) and, where the k-th energy is tied, on the row/index among
// the tied entries; keys are unique (a row is walked once, an index occurs
// once), so exactly min(k, candidates) entries are kept.
#include "device_energy.h"
#include "kcommon.h"
#include "kernels.h"

namespace qk {

namespace {

constexpr int kSelThreads = 1024;   // also the largest k

struct SelArgs {
    const int32_t *E;          // dense candidates [0, *count * mult)
    const uint64_t *R;
    const int32_t *count;
    uint32_t mult;
    int k;
    int32_t *oE;               // [k] output, sorted by (E, R)
    uint64_t *oR;
    int32_t *oCount;
    int32_t *clear;            // set to 0 when done (a later kernel's counter), or null
};

__device__ __forceinline__ uint32_t ukey(int32_t e) { return uint32_t(e) ^ 0x80000000u; }

__device__ __forceinline__ bool key_less(int32_t ea, uint64_t ra, int32_t eb, uint64_t rb)
{
    return ea < eb || (ea == eb && ra < rb);
}

// Visit every candidate: f(E, R).
template <typename F>
__device__ __forceinline__ void for_valid(const SelArgs &a, uint32_t N, F &&f)
{
    for (uint32_t x = threadIdx.x; x < N; x += kSelThreads) f(a.E[x], a.R[x]);
}

// Bin of the histogram where the running count reaches `need`.
__device__ void pick_bin(const uint32_t *hist, uint32_t need, uint32_t *bin, uint32_t *rest,
                         uint32_t *inbin)
{
    uint32_t cum = 0;
    for (uint32_t b = 0; b < 256; b++) {
        if (cum + hist[b] >= need) {
            *bin = b;
            *rest = need - cum;
            *inbin = hist[b];
            return;
        }
        cum += hist[b];
    }
    *bin = 255;      // unreachable when need <= total
    *rest = 0;
    *inbin = 0;
}

__global__ __launch_bounds__(kSelThreads) void topk_select_kernel(SelArgs a)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t sh_total, sh_pos, sh_bin, sh_rest, sh_in;
    __shared__ int32_t sE[kSelThreads];
    __shared__ uint64_t sR[kSelThreads];
    const uint32_t tid = threadIdx.x;
    const uint32_t k = uint32_t(a.k);

    if (tid == 0) {
        sh_total = uint32_t(*a.count) * a.mult;
        sh_pos = 0;
    }
    __syncthreads();
    const uint32_t total = sh_total;

    bool take_all = total <= k;
    uint32_t uk = 0xFFFFFFFFu;      // energy key of the k-th entry
    bool all_eq = true;             // take every entry whose key equals uk
    uint64_t rk = ~0ull;            // else those with R <= rk
    if (!take_all) {
        uint32_t prefix = 0, mask = 0, need = k;
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (uint32_t b = tid; b < 256; b += kSelThreads) hist[b] = 0;
            __syncthreads();
            for_valid(a, total, [&](int32_t e, uint64_t) {
                const uint32_t u = ukey(e);
                if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1u);
            });
            __syncthreads();
            if (tid == 0) pick_bin(hist, need, &sh_bin, &sh_rest, &sh_in);
            __syncthreads();
            prefix |= sh_bin << shift;
            mask |= 255u << shift;
            need = sh_rest;
            __syncthreads();
        }
        uk = prefix;
        all_eq = need == sh_in;     // every entry with energy key uk is kept
        if (!all_eq) {
            uint64_t rprefix = 0, rmask = 0;
            for (int shift = 56; shift >= 0; shift -= 8) {
                for (uint32_t b = tid; b < 256; b += kSelThreads) hist[b] = 0;
                __syncthreads();
                for_valid(a, total, [&](int32_t e, uint64_t r) {
                    if (ukey(e) == uk && (r & rmask) == rprefix)
                        atomicAdd(&hist[uint32_t(r >> shift) & 255u], 1u);
                });
                __syncthreads();
                if (tid == 0) pick_bin(hist, need, &sh_bin, &sh_rest, &sh_in);
                __syncthreads();
                rprefix |= uint64_t(sh_bin) << shift;
                rmask |= uint64_t(255) << shift;
                need = sh_rest;
                __syncthreads();
            }
            rk = rprefix;
        }
    }
    // compaction into LDS (at most k entries)
    for_valid(a, total, [&](int32_t e, uint64_t r) {
        const uint32_t u = ukey(e);
        if (take_all || u < uk || (u == uk && (all_eq || r <= rk))) {
            const uint32_t p = atomicAdd(&sh_pos, 1u);
            if (p < k) {
                sE[p] = e;
                sR[p] = r;
            }
        }
    });
    __syncthreads();
    const uint32_t cnt = min(sh_pos, k);
    // bitonic sort of the kept entries by (E, R), padded to a power of two
    uint32_t P = 1;
    while (P < cnt) P <<= 1;
    if (tid >= cnt && tid < P) {
        sE[tid] = INT32_MAX;
        sR[tid] = ~0ull;
    }
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t st = size >> 1; st > 0; st >>= 1) {
            const uint32_t j = tid ^ st;
            if (tid < P && j > tid) {
                const bool asc = (tid & size) == 0;
                const bool jl = key_less(sE[j], sR[j], sE[tid], sR[tid]);
                if (jl == asc) {
                    const int32_t te = sE[tid];
                    const uint64_t tr = sR[tid];
                    sE[tid] = sE[j];
                    sR[tid] = sR[j];
                    sE[j] = te;
                    sR[j] = tr;
                }
            }
            __syncthreads();
        }
    }
    if (tid < cnt) {
        a.oE[tid] = sE[tid];
        a.oR[tid] = sR[tid];
    }
    if (tid == 0) {
        *a.oCount = int32_t(cnt);
        if (a.clear) *a.clear = 0;
    }
}

// The walk lists, compacted: entries with E <= *bound of every wave's list,
// appended densely (one wave per list, wave-aggregated slots).
__global__ __launch_bounds__(256) void topk_compact_kernel(const int32_t *__restrict__ E,
                                                           const uint64_t *__restrict__ R,
                                                           const int32_t *__restrict__ listCount,
                                                           int nlists, int stride,
                                                           const int32_t *__restrict__ bound,
                                                           int32_t *__restrict__ oE,
                                                           uint64_t *__restrict__ oR,
                                                           int32_t *__restrict__ oN)
{
    const int lane = int(threadIdx.x) & (kWave - 1);
    const int list = int(blockIdx.x) * (256 / kWave) + int(threadIdx.x) / kWave;
    if (list >= nlists) return;
    const int32_t bnd = *bound;
    const int c = listCount[list];
    for (int p0 = 0; p0 < c; p0 += kWave) {
        const int p = p0 + lane;
        const size_t x = size_t(list) * size_t(stride) + size_t(p);
        const bool keep = p < c && E[x] <= bnd;
        const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
        if (!m) continue;
        int base = 0;
        if (lane == 0) base = atomicAdd(oN, int(__builtin_popcountll(m)));
        base = __builtin_amdgcn_readfirstlane(base);
        if (keep) {
            const int rank = int(__builtin_popcountll(m & ((1ull << lane) - 1)));
            oE[base + rank] = E[x];
            oR[base + rank] = R[x];
        }
    }
}

// Step 3: block b rescans chunk rows[b] (if b < *rowCount) and appends its
// states with E <= the largest selected chunk key to (stE, stI), densely
// (wave-aggregated slots counted in *stCount, zeroed by the chunk select).
// With fewer than k chunks selected (the instance has fewer than k chunks)
// the k-th smallest state may lie above every chunk minimum, so every state
// of every chunk is kept: at most rc << B < k << B entries.
__global__ __launch_bounds__(256) void topk_rescan_kernel(const Inst *__restrict__ inst,
                                                          const uint64_t *__restrict__ rows,
                                                          const int32_t *__restrict__ rowE,
                                                          const int32_t *__restrict__ rowCount,
                                                          int k,
                                                          int32_t *__restrict__ stE,
                                                          uint64_t *__restrict__ stI,
                                                          int32_t *__restrict__ stCount)
{
    __shared__ int64_t red[256];
    const Inst I = *inst;
    const int n = I.n, A = I.A, B = I.B;
    const uint32_t NS = 1u << B;
    const uint32_t b = blockIdx.x;
    const int32_t rc = *rowCount;
    if (int32_t(b) >= rc) return;
    // rows are sorted by (key, row)
    const int32_t bound = rc < k ? INT32_MAX : rowE[rc - 1];
    const int lane = int(threadIdx.x) & (kWave - 1);
    const uint64_t row = rows[b];
    // E_p(row) = sum over set prefix bits i <= j of T[i][j]; prefix variable
    // v is bit A-1-v of the U_A row.
    int64_t part = 0;
    for (int i = int(threadIdx.x); i < A; i += int(blockDim.x)) {
        if (!((row >> (A - 1 - i)) & 1)) continue;
        for (int j = i; j < A; j++)
            if ((row >> (A - 1 - j)) & 1) part += I.T[i * n + j];
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    const int32_t Ep = int32_t(red[0]);
    // state (row, s) of energy e: kept when at most the bound (the whole
    // wave calls this together)
    auto offer = [&](int32_t e, uint32_t s) {
        const bool keep = e <= bound;
        const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
        if (!m) return;
        int base = 0;
        if (lane == 0) base = atomicAdd(stCount, int(__builtin_popcountll(m)));
        base = __builtin_amdgcn_readfirstlane(base);
        if (keep) {
            const int p = base + int(__builtin_popcountll(m & ((1ull << lane) - 1)));
            stE[p] = e;
            stI[p] = (row << B) | s;
        }
    };
    // NS (and NS / 2) is a multiple of 64: every lane of a wave that enters
    // runs each pass
    if (I.packed) {
        // the walk's own arithmetic: the packed words of the chunk summed mod
        // 2^32, then both 16-bit halves decoded (columns c and c + NS / 2)
        const uint32_t NW = NS / 2;
        const int32_t off = kPackBias + I.pack_shift;
        for (uint32_t c = threadIdx.x; c < NW; c += blockDim.x) {
            uint32_t w = uint32_t(I.EB[c]);
            for (int v = 0; v < A; v++)
                if ((row >> (A - 1 - v)) & 1) w += uint32_t(I.M[uint32_t(v) * NW + c]);
            offer(Ep + int32_t(w & 0xffffu) - off, c);
            offer(Ep + int32_t(w >> 16) - off, c + NW);
        }
    } else {
        for (uint32_t s = threadIdx.x; s < NS; s += blockDim.x) {
            int32_t e = Ep - I.pack_shift + I.EB[s];   // E_s carries the walk's shift
            for (int v = 0; v < A; v++)
                if ((row >> (A - 1 - v)) & 1) e += I.M[uint32_t(v) * NS + s];
            offer(e, s);
        }
    }
}

// Step 3 for direct instances: every state.
__global__ __launch_bounds__(256) void topk_direct_kernel(const Inst *__restrict__ inst,
                                                          int32_t *__restrict__ stE,
                                                          uint64_t *__restrict__ stI,
                                                          int32_t *__restrict__ segCount)
{
    const Inst I = *inst;
    const uint32_t N = 1u << I.n;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < N; r += gridDim.x * blockDim.x) {
        stE[r] = int32_t(energy_int(I.T, I.n, r));
        stI[r] = r;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) segCount[0] = int32_t(N);
}

// Step 5: verify, rescore, order; one block of k (<= 1024) threads.
__global__ __launch_bounds__(kSelThreads) void topk_final_kernel(
    const Inst *__restrict__ inst, const int32_t *__restrict__ selE,
    const uint64_t *__restrict__ selR, const int32_t *__restrict__ selCount, int k,
    TopkState *__restrict__ out, FinalRes *__restrict__ best)
{
    __shared__ double sF[kSelThreads];
    __shared__ uint64_t sI[kSelThreads];
    __shared__ int64_t sE[kSelThreads];
    __shared__ int32_t sh_bad;
    const Inst I = *inst;
    const uint32_t tid = threadIdx.x;
    const int cnt = *selCount;
    if (tid == 0) sh_bad = 0;
    __syncthreads();
    if (int(tid) < cnt) {
        const uint64_t idx = selR[tid];
        const int64_t e = selE[tid];
        if (energy_int(I.T, I.n, idx) != e) atomicOr(&sh_bad, 1);
        sE[tid] = e;
        sI[tid] = idx;
        sF[tid] = I.Qf ? energy_f64(I.Qf, I.n, idx) : double(e);
    }
    __syncthreads();
    if (I.Qf) {
        // the integer order is exact for the scaled energies; report the
        // float64 energies in their own (E64, index) order
        uint32_t P = 1;
        while (P < uint32_t(cnt)) P <<= 1;
        if (int(tid) >= cnt && tid < P) {
            sF[tid] = __builtin_huge_val();
            sI[tid] = ~0ull;
            sE[tid] = 0;
        }
        __syncthreads();
        for (uint32_t size = 2; size <= P; size <<= 1) {
            for (uint32_t st = size >> 1; st > 0; st >>= 1) {
                const uint32_t j = tid ^ st;
                if (tid < P && j > tid) {
                    const bool asc = (tid & size) == 0;
                    const bool jl = sF[j] < sF[tid] || (sF[j] == sF[tid] && sI[j] < sI[tid]);
                    if (jl == asc) {
                        const double tf = sF[tid];
                        const uint64_t ti = sI[tid];
                        const int64_t te = sE[tid];
                        sF[tid] = sF[j];
                        sI[tid] = sI[j];
                        sE[tid] = sE[j];
                        sF[j] = tf;
                        sI[j] = ti;
                        sE[j] = te;
                    }
                }
                __syncthreads();
            }
        }
    }
    if (int(tid) < cnt && int(tid) < k) {
        TopkState o;
        o.E = sE[tid];
        o.E64 = sF[tid];
        o.index = sI[tid];
        out[tid] = o;
    }
    if (tid == 0) {
        FinalRes r;
        const int32_t status = sh_bad ? 3 : (cnt < k ? 4 : 0);
        r.E = cnt > 0 ? sE[0] : 0;
        r.index = cnt > 0 ? sI[0] : 0;
        r.E64 = cnt > 0 ? sF[0] : 0.0;
        r.status = status;
        r.pad = 0;
        *best = r;
    }
}

// ---------------------------------------------------------------- seed
// Upper bound of the k-th smallest chunk key, set as the shared bound before
// the walk (which then only lowers it).  Chunks of distinct prefix rows are
// distinct, and a state's energy bounds its own chunk's key from above, so
// the k-th smallest energy over states with k or more distinct prefix rows
// bounds the k-th smallest chunk key.  The states: a local minimum x* of
// eight greedy descents and the states that differ from it in one to four
// prefix variables (the first kSeedStates in order of the number of flips,
// each group in colex order).  Their energies follow from x*'s single-flip
// changes d_i and the couplings: flipping the set F changes E by
//   sum_{i in F} d_i + sum_{i<j in F} s_i s_j T_ij,   s_i = 1 - 2 x_i.
constexpr int kSeedStates = 4096;
constexpr int kSeedThreads = 256;

__device__ __forceinline__ int64_t binom_small(int v, int r)   // C(v, r), r <= 4
{
    if (v < r) return 0;
    int64_t c = 1;
    for (int t = 0; t < r; t++) c = c * (v - t) / (t + 1);
    return c;
}

__global__ __launch_bounds__(kSeedThreads) void topk_seed_kernel(const Inst *__restrict__ inst,
                                                                 int32_t *gthr, int k)
{
    const Inst &I = *inst;
    const int n = I.n, A = I.A;
    const int32_t *T = I.T;
    const int tid = int(threadIdx.x), lane = tid % kWave, wave = tid / kWave;
    __shared__ int32_t wE[kSeedThreads / kWave];
    __shared__ uint64_t wX[kSeedThreads / kWave];
    __shared__ int32_t d[kWave];
    __shared__ int32_t sg[kWave];
    __shared__ int32_t Ec[kSeedStates];
    __shared__ int64_t sBest;
    __shared__ uint64_t sXm;
    __shared__ uint32_t sCount;

    // 1. the best local minimum of eight descents (two per wave)
    int32_t bE = kNoEnergy;
    uint64_t bX = 0;
    for (int rep = 0; rep < 2; rep++) {
        int32_t E;
        uint64_t xm;
        greedy_descent(T, n, uint32_t(wave) * 2u + uint32_t(rep), E, xm);
        if (E < bE || (E == bE && xm < bX)) {
            bE = E;
            bX = xm;
        }
    }
    if (lane == 0) {
        wE[wave] = bE;
        wX[wave] = bX;
    }
    __syncthreads();
    if (tid == 0) {
        int32_t e = wE[0];
        uint64_t x = wX[0];
        for (int w = 1; w < kSeedThreads / kWave; w++)
            if (wE[w] < e || (wE[w] == e && wX[w] < x)) {
                e = wE[w];
                x = wX[w];
            }
        sBest = e;
        sXm = x;
    }
    __syncthreads();
    const uint64_t xm = sXm;
    // 2. single-flip changes and signs at x*, one thread per variable
    if (tid < n) {
        const int xl = int((xm >> tid) & 1);
        int32_t f = T[tid * n + tid];
        for (int j = 0; j < n; j++)
            if (j != tid && ((xm >> j) & 1)) f += j < tid ? T[j * n + tid] : T[tid * n + j];
        d[tid] = xl ? -f : f;
        sg[tid] = xl ? -1 : 1;
    }
    // 3. the states with 0..4 prefix variables flipped
    int64_t groups[5];
    int64_t total = 0;
    for (int p = 0; p <= 4; p++) {
        groups[p] = binom_small(A, p);
        total += groups[p];
    }
    const int M = int(total < kSeedStates ? total : kSeedStates);
    if (M < k) return;   // fewer distinct rows than k: no bound
    __syncthreads();
    for (int c = tid; c < M; c += kSeedThreads) {
        int p = 0;
        int64_t rank = c;
        while (rank >= groups[p]) rank -= groups[p++];
        int v[4];
        for (int r = p; r >= 1; r--) {   // colex unranking of the p-subset
            int x = r - 1;
            while (binom_small(x + 1, r) <= rank) x++;
            rank -= binom_small(x, r);
            v[r - 1] = x;
        }
        int64_t e = sBest;
        for (int a = 0; a < p; a++) {
            e += d[v[a]];
            for (int b = 0; b < a; b++) {
                const int i = v[b], j = v[a];   // i < j
                e += int64_t(sg[i] * sg[j]) * T[i * n + j];
            }
        }
        Ec[c] = int32_t(e);
    }
    __syncthreads();
    // 4. the k-th smallest of the M energies: the least value v with at
    //    least k energies <= v (bisection on v with block-wide counts)
    int64_t lo = INT32_MAX, hi = INT32_MIN;
    for (int c = 0; c < M; c++) {   // every thread the same bounds
        lo = min(lo, int64_t(Ec[c]));
        hi = max(hi, int64_t(Ec[c]));
    }
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (tid == 0) sCount = 0;
        __syncthreads();
        uint32_t cnt = 0;
        for (int c = tid; c < M; c += kSeedThreads) cnt += Ec[c] <= mid ? 1u : 0u;
        atomicAdd(&sCount, cnt);
        __syncthreads();
        const uint32_t total_le = sCount;
        __syncthreads();
        if (total_le >= uint32_t(k)) hi = mid;
        else lo = mid + 1;
    }
    if (tid == 0) atomicMin(gthr, int32_t(lo));
}

}  // namespace

hipError_t launch_topk_seed(const Inst *d_inst, int32_t *d_gthr, int k, hipStream_t stream)
{
    if (k < 2 || k > kSeedStates) return hipErrorInvalidValue;
    hipLaunchKernelGGL(topk_seed_kernel, dim3(1), dim3(kSeedThreads), 0, stream, d_inst, d_gthr, k);
    return hipGetLastError();
}

hipError_t launch_topk_finish(const Inst *d_inst, const Inst &hI, const TopkBufs &buf, int k,
                              FinalRes *d_best, hipStream_t stream)
{
    if (k < 2 || k > kSelThreads) return hipErrorInvalidValue;
    SelArgs st{};
    if (hI.direct) {
        const uint32_t N = 1u << hI.n;
        const uint32_t blocks = (N + 255) / 256;
        hipLaunchKernelGGL(topk_direct_kernel, dim3(blocks), dim3(256), 0, stream, d_inst, buf.stE,
                           buf.stI, buf.segCount);
        st.count = buf.segCount;     // 2^n
        st.mult = 1;
    } else {
        // the lists' entries at or below the final shared bound, densely
        const int lists_per_block = 256 / kWave;
        const int blocks = (buf.waves + lists_per_block - 1) / lists_per_block;
        if (blocks > 0)
            hipLaunchKernelGGL(topk_compact_kernel, dim3(blocks), dim3(256), 0, stream,
                               buf.walk.listE, buf.walk.listR, buf.walk.listCount, buf.waves, k,
                               buf.walk.gthr, buf.candE, buf.candR, buf.candN);
        SelArgs ch{};
        ch.E = buf.candE;
        ch.R = buf.candR;
        ch.count = buf.candN;
        ch.mult = 1;
        ch.k = k;
        ch.oE = buf.chunkE;
        ch.oR = buf.chunkR;
        ch.oCount = buf.chunkCount;
        ch.clear = buf.segCount;     // [0]: the rescan's state counter
        hipLaunchKernelGGL(topk_select_kernel, dim3(1), dim3(kSelThreads), 0, stream, ch);
        hipLaunchKernelGGL(topk_rescan_kernel, dim3(k), dim3(256), 0, stream, d_inst, buf.chunkR,
                           buf.chunkE, buf.chunkCount, k, buf.stE, buf.stI, buf.segCount);
        st.count = buf.segCount;     // states kept by the rescan, densely
        st.mult = 1;
    }
    st.E = buf.stE;
    st.R = buf.stI;
    st.k = k;
    st.oE = buf.selE;
    st.oR = buf.selR;
    st.oCount = buf.selCount;
    hipLaunchKernelGGL(topk_select_kernel, dim3(1), dim3(kSelThreads), 0, stream, st);
    hipLaunchKernelGGL(topk_final_kernel, dim3(1), dim3(kSelThreads), 0, stream, d_inst, buf.selE,
                       buf.selR, buf.selCount, k, buf.out, d_best);
    return hipGetLastError();
}

}  // namespace qk

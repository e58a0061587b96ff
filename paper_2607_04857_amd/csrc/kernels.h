// kernels.h -- device data layout and kernel launchers of the solver.
//
// Layout in HBM per instance (all int32 unless noted; built by table_kernel):
//   T   [n][n]        folded upper-triangular matrix (input of the table build)
//   M   [A][2^B]      interaction rows M_int[v][s] = sum over set suffix bits t
//                     of T[v][A+t] (Sec. II-C: M_int = Q_ps U_B^T), column s
//                     stored at s = j*64 + lane so lane `lane` owns columns
//                     {j*64 + lane}, j < 2^B/64 (column-wise split, Sec. III-C.2)
//   EB  [2^B]         suffix energies E_s(U_B) (Sec. III-A, preprocessing 2)
//                     Packed instances (tiers 4, 5) store 2^(B-1) words per row:
//                     word c holds column c in its low 16 bits and column
//                     c + 2^(B-1) (suffix variable A set) in its high 16
//                     bits, EB biased by kPackBias in each half, so one
//                     32-bit add moves both energies (see kPackSumLimit)
//   S   [A][64]       S[w][l] = T[min(l,w)][max(l,w)] for l != w < A, else 0:
//                     the prefix couplings, one lane per variable
//   K   [6][32]+[12]  (all instances' K tables are contiguous) tier-2 bound
//                     constants per 64-step super-block offset o and table
//                     (0: o < 32; 1: o >= 32, level-5 bit rising; 2: o >= 32,
//                     falling), entry o mod 32: rows 0..2 hold C2 = ELOW + D,
//                     rows 3..5 hold D, where D is the minimum over all 2^B
//                     columns of E_sd(o) - E_sd(super-block start) and ELOW
//                     the low-low coupling energy of the low pattern at o;
//                     then the minima of C2 over each bound-test segment
//                     (kc2min_slot: per table for 32-step segments, per
//                     table half for 16-step ones; 12 entries); then
//                     SL[64][5]: SL[w][t] = coupling of prefix variable w
//                     with the low variable A-1-t (0 when equal), so a flip
//                     of w moves the low fields by scalar loads only
//   Qf  [n][n] fp32   caller's float32 Q (fp32 instances only, for rescoring)
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qk {

constexpr int kWave = 64;
constexpr int kSuperLog = 6;          // unrolled super-block: 64 Gray steps
constexpr int kLowLevels = 5;         // Gray levels with static patterns in a super-block
constexpr int kPatterns = 1 << kLowLevels;
constexpr int kSegSteps = 32;         // steps per tier-2 bound-test segment (measured
                                      // 3.7% faster than 16 at n = 44)
constexpr int kSegStepsTopk = 16;     // tier 3, whose looser threshold passes more often
static_assert(kPatterns == 32, "bound-test segments of 32 (a table) or 16 steps");
constexpr int kKC2Min = 6 * kPatterns;   // min of C2 per (table, segment)
constexpr int kKBound = kKC2Min + 12;    // bound constants at the head of a K table
// Slot of the minimum of C2 over segment h of table tab: 32-step segments
// (a whole table) at kKC2Min + tab, 16-step ones at kKC2Min + 3 + 2 tab + h % 2.
__host__ __device__ constexpr int kc2min_slot(int seg_steps, int tab, int h)
{
    return seg_steps == 32 ? kKC2Min + tab : kKC2Min + 3 + 2 * tab + (h & 1);
}
constexpr int kKTable = kKBound + kLowLevels * kWave;  // + SL[w][t], t < kLowLevels
constexpr int kMaxVgprLevels = 12;    // at most Gray levels 0..11 keep their M_int row in VGPRs
constexpr int32_t kNoEnergy = 1 << 30;  // above every energy the walk can meet
constexpr int kMaxVars = 60;          // largest n the planner accepts
constexpr int kMaxPrefixRows = 60 - 6;   // A = n - B <= 60 - 6
// Packed walk (tiers 4 and 5, the int16 energies of Sec. IV-B "Data types"
// at two per 32-bit word).  Word = (E_lo + c + kPackBias) + (E_hi + c +
// kPackBias) 2^16 and a row word = m_lo + m_hi 2^16 (mod 2^32), with c the
// instance's shift below: the map is additive mod 2^32, so a
// 32-bit add of a row word adds m_lo and m_hi to the two halves however the
// intermediate carries fall, and a word decodes exactly whenever both biased
// halves lie in [0, 2^16).  The planner proves every chunk energy E_sd + c
// (c = Inst::pack_shift, a constant per instance) a signed 16-bit value from
// the exact extremes of E_sd over all prefixes and columns, and picks c so
// that the least biased half is 0.
constexpr int32_t kPackBias = 1 << 15;
constexpr int64_t kPackSumLimit = (int64_t(1) << 15) - 1;

struct ItemRes;

// An instance whose Q is prepared on the device (lone solve of a device
// pointer): the preparation's outcome, written by prepare_kernel.
constexpr int64_t kExactSumLimit = (int64_t(1) << 30) - 1;   // sum |T| bound of the int32 walk
constexpr int32_t kPrepOverflow = 1;    // int32 input with sum |T| above kExactSumLimit
constexpr int32_t kPrepNonFinite = 2;   // float32 input with a NaN or Inf
constexpr int32_t kPrepInternal = 3;    // scaled float32 matrix above the bound
struct PrepOut {
    int32_t status;      // 0, or kPrepOverflow / kPrepNonFinite / kPrepInternal
    int32_t p;           // fixed-point exponent (float32 input), else 0
    int64_t sum_abs;     // sum of |T_ij|, i <= j, of the int32 matrix solved
    double eps_q;        // per-state quantisation bound (float32 input), else 0
    int64_t hist_lo;     // top-k histogram: energy of bin 0's lower edge ...
    int32_t hist_shift;  // ... and the bin shift
    int32_t pad;
};

struct Inst {
    const int32_t *T;
    int32_t *M;
    int32_t *EB;
    int32_t *S;
    int32_t *K;            // this instance's K table (kslot-th table of the K array)
    const float *Qf;
    ItemRes *res;          // this launch's item results: item g of the launch
                           // (item_begin <= g < item_end) that found a candidate
                           // writes res[g - item_begin] ...
    uint32_t *bits;        // ... and sets bit bit0 + (g - item_begin) of the
                           // instance's item bitmap (bit q <-> res record q of
                           // the instance; cleared by the table build), so the
                           // finish reads only records that were written
    uint64_t bit0;
    int n, A, B, L;
    int direct;            // 1: no walk, direct evaluation of all 2^n states
    int kslot;             // index of the K table in the launch's K array
    int packed;            // 1: M and EB in the packed 16-bit layout (tiers 4, 5)
    int32_t pack_shift;    // c added to every chunk energy in EB and taken
                           // off the prefix energy: tiers 4, 5 make every
                           // E_sd + c a signed 16-bit value, the int32 walk
                           // makes it non-negative (written by prepare_kernel
                           // for a device-prepared instance)
    uint64_t item_begin;   // this launch's walk-item range [item_begin, item_end)
    uint64_t item_end;
    uint64_t item_local0;  // the instance's own item number of launch item item_begin
    uint64_t n_items;      // item records of the instance (res[0 .. n_items), bitmap
                           // words bits[0 .. ceil(n_items / 32)))
    int32_t *gbest;        // best energy any wave has found for the instance
                           // (kNoEnergy from the table build on)
    const PrepOut *prep;   // device-prepared instance: its preparation (an error
                           // makes the walk skip all items), else null
};

struct ItemRes {
    int32_t E;         // best energy accepted inside the item
    int32_t found;     // 1 (only items that found a candidate write a record)
    uint64_t row;      // prefix row (U_A row) of that chunk
};

// Top-k (k > 1) state of one walk launch over a single instance.  Each
// wave keeps, in listE / listR (its slot of k entries), the k smallest chunk
// keys (E_p + min over the chunk, prefix row) it has met; a chunk can belong to the instance's k smallest
// chunks only if its minimum is at most the largest E of any full list, so
// waves share that bound through gthr (atomic min).
struct TopkWalk {
    int32_t *listE;      // [waves][k] chunk minima
    uint64_t *listR;     // [waves][k] prefix rows of those chunks
    int32_t *listCount;  // [waves] entries used (written by every wave on exit)
    int32_t *gthr;       // shared bound, kNoEnergy before the walk
    uint32_t *hist;      // [kTopkBins] keys entered into any list, by energy bin (zeroed)
    int32_t *lowbin;     // lowest non-empty bin (kTopkBins before the walk)
    int64_t hist_lo;     // energy of bin 0's lower edge (-sum|T|)
    int hist_shift;      // bin = (E - hist_lo) >> hist_shift
    int k;
    const PrepOut *prep; // device-prepared instance: hist_lo and hist_shift come
                         // from here instead (null otherwise)
};
constexpr int kTopkBins = 16384;

// One state of a top-k answer; the same layout as qubo_state_t.
struct TopkState {
    int64_t E;           // exact integer energy
    double E64;          // float64 rescore (fp32) or (double)E
    uint64_t index;      // U_N row
};

// Device buffers of the top-k finish of a single instance.
struct TopkBufs {
    TopkWalk walk;
    int waves;           // lists in walk.listE (walked instances)
    int32_t *candE;      // [waves * k] list entries <= the final bound, dense ...
    uint64_t *candR;
    int32_t *candN;      // [1] their number (zero before the finish)
    int32_t *chunkE;     // [k] the k smallest chunk keys ...
    uint64_t *chunkR;    // [k] ... and their prefix rows
    int32_t *chunkCount; // [1] chunks selected (min(k, chunks met))
    int32_t *stE;        // [k << B] (or [2^n] direct) candidate state energies
    uint64_t *stI;       // same, U_N rows
    int32_t *segCount;   // [0]: states kept by the rescan (2^n when direct)
    int32_t *selE;       // [k] the k smallest states, sorted by (E, index)
    uint64_t *selR;
    int32_t *selCount;   // [1]
    TopkState *out;      // [k] answer (fp32: sorted by (E64, index))
};

struct FinalRes {
    int64_t E;         // exact integer energy of the answer
    uint64_t index;    // U_N row of the answer
    double E64;        // float64 rescore from Qf (fp32 instances)
    int32_t status;    // 0 ok, nonzero: self-check failure
    int32_t pad;
};

// Fold, check and (float32) scale the caller's device matrix dQ (n x n,
// row-major, int32 or float32) into the instance's upper-triangular int32 T
// (d_T, n x n), exactly as the host planner does, and write the outcome to
// *d_prep and the walk's chunk-energy shift to d_inst->pack_shift (the
// descriptor's split A, B already set; int32 walk only).  On an input error
// T is left zero and the status says why.
hipError_t launch_prepare(const void *dQ, int n, int is_fp32, int32_t *d_T, PrepOut *d_prep,
                          Inst *d_inst, hipStream_t stream);

// Builds M, EB, S, K for every instance, clears each instance's item bitmap
// and shared best, and zeroes n_counters item counters (for a device-prepared
// instance whose preparation failed, the counters are set past every item).
hipError_t launch_tables(const Inst *d_insts, int n_inst, int max_A, unsigned long long *d_counters,
                         int n_counters, hipStream_t stream);

// Persistent Gray walk over all items; `waves` resident wavefronts.  d_k is
// the contiguous array of K tables (instance i's at insts[i].kslot*kKTable).
// Variant: mcols words per lane (B = 6 + log2 mcols, 7 + log2 mcols for
// tiers 4 and 5), the M_int rows of Gray levels below vgpr_levels cached in
// VGPRs (higher ones from L2), tier.
// Tiers 3 and 5 (top-k lists) need `tk` and exactly one instance; tiers 1,
// 2 and 4 ignore it (may be null).
hipError_t launch_walk(int mcols, int vgpr_levels, int tier, const Inst *d_insts, int n_inst,
                       uint64_t total_items, unsigned long long *d_counter, const int32_t *d_k,
                       int waves, hipStream_t stream, const TopkWalk *tk = nullptr);

// Whether a (mcols, vgpr_levels) walk variant is compiled in, and whether
// its packed form (tiers 4 and 5: 2 mcols 64 suffix columns) is.
bool walk_variant_exists(int mcols, int vgpr_levels);
bool walk_packed_exists(int mcols, int vgpr_levels);

// Resident walk wavefronts per CU for a variant (occupancy query, >= 1);
// topk_k > 1 accounts for tier 3's LDS list.
int walk_occupancy(int mcols, int vgpr_levels, int tier, int topk_k = 0);

// LDS bytes of one tier-3 wave's list scalars (its k entries are in listE /
// listR in global memory).
constexpr int kTopkMetaWords = 13;  // 64-bit words of list scalars
__host__ __device__ inline size_t topk_lds_bytes()
{
    return size_t(kTopkMetaWords) * 8;
}

// Seeds the shared top-k bound *d_gthr of one walked instance before its
// walk: the k-th smallest energy of up to 4096 states with distinct prefix
// rows near a local minimum (every walked chunk must be in the walk: full
// item range only).  Leaves *d_gthr unchanged when the instance has fewer
// such states than k.
hipError_t launch_topk_seed(const Inst *d_inst, int32_t *d_gthr, int k, hipStream_t stream);

// Top-k finish of one instance (descriptor d_inst, host copy hI): select the
// k smallest chunks of the walk lists, rescan them (or, direct, evaluate all
// 2^n states), select and sort the k smallest states, verify their energies
// and write buf.out and *d_best (status 3: an energy did not verify; 4:
// fewer than k states).
hipError_t launch_topk_finish(const Inst *d_inst, const Inst &hI, const TopkBufs &buf, int k,
                              FinalRes *d_best, hipStream_t stream);

// Per-instance reduction of item results (insts[i].res[0..n_items)), argmin
// rescan (or direct evaluation for tiny n) and float64 rescoring; one
// FinalRes per descriptor.
hipError_t launch_finish(const Inst *d_insts, int n_inst, FinalRes *d_out, hipStream_t stream);

}  // namespace qk

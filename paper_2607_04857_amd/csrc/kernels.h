// kernels.h -- device data layout and kernel launchers of the solver.
//
// Layout in HBM per instance (all int32 unless noted; built by table_kernel):
//   T   [n][n]        folded upper-triangular matrix (input of the table build)
//   M   [A][2^B]      interaction rows M_int[v][s] = sum over set suffix bits t
//                     of T[v][A+t] (Sec. II-C: M_int = Q_ps U_B^T), column s
//                     stored at s = j*64 + lane so lane `lane` owns columns
//                     {j*64 + lane}, j < 2^B/64 (column-wise split, Sec. III-C.2)
//   EB  [2^B]         suffix energies E_s(U_B) (Sec. III-A, preprocessing 2)
//   S   [A][64]       S[w][l] = T[min(l,w)][max(l,w)] for l != w < A, else 0:
//                     the prefix couplings, one lane per variable
//   K   [6][16]       (all instances' K tables are contiguous) tier-2 bound constants per super-block offset o and
//                     table (0: o < 16; 1: o >= 16, level-4 bit rising;
//                     2: o >= 16, falling): rows 0..2 hold C2 = ELOW + D,
//                     rows 3..5 hold D, where D is the minimum over all 2^B
//                     columns of E_sd(o) - E_sd(super-block start) and ELOW the
//                     low-low coupling energy of the low pattern at o;
//                     then SL[64][4]: SL[w][t] = coupling of prefix variable w
//                     with the low variable A-1-t (0 when equal), so a flip of
//                     w moves the low fields by scalar loads only
//   Qf  [n][n] fp32   caller's float32 Q (fp32 instances only, for rescoring)
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qk {

constexpr int kWave = 64;
constexpr int kSuperLog = 5;          // unrolled super-block: 32 Gray steps
constexpr int kLowLevels = 4;         // Gray levels with static patterns in a super-block
constexpr int kPatterns = 1 << kLowLevels;
constexpr int kKBound = 6 * kPatterns;   // bound constants at the head of a K table
constexpr int kKTable = kKBound + 4 * kWave;  // + SL[w][t], t < 4: ints per K table
constexpr int kMaxVgprLevels = 12;    // at most Gray levels 0..11 keep their M_int row in VGPRs
constexpr int32_t kNoEnergy = 1 << 30;  // above every energy the walk can meet

struct ItemRes;

struct Inst {
    const int32_t *T;
    int32_t *M;
    int32_t *EB;
    int32_t *S;
    int32_t *K;            // this instance's K table (kslot-th table of the K array)
    const float *Qf;
    ItemRes *res;          // per-item results of this instance, by local item index
    int n, A, B, L;
    int direct;            // 1: no walk, direct evaluation of all 2^n states
    int kslot;             // index of the K table in the launch's K array
    uint64_t item_begin;   // this launch's walk-item range [item_begin, item_end)
    uint64_t item_end;
    uint64_t item_local0;  // local index of the instance's item number item_begin
    uint64_t n_items;      // the instance's total items, 2^(A-L)
};

struct ItemRes {
    int32_t E;         // best energy accepted inside the item (kNoEnergy: none)
    int32_t found;
    uint64_t row;      // prefix row (U_A row) of that chunk
};

struct FinalRes {
    int64_t E;         // exact integer energy of the answer
    uint64_t index;    // U_N row of the answer
    double E64;        // float64 rescore from Qf (fp32 instances)
    int32_t status;    // 0 ok, nonzero: self-check failure
    int32_t pad;
};

// Builds M, EB, S, K for every instance and zeroes n_counters item counters.
hipError_t launch_tables(const Inst *d_insts, int n_inst, int max_A, unsigned long long *d_counters,
                         int n_counters, hipStream_t stream);

// Persistent Gray walk over all items; `waves` resident wavefronts.  d_k is
// the contiguous array of K tables (instance i's at insts[i].kslot*kKTable).
// Variant: mcols columns per lane (B = 6 + log2 mcols), the M_int rows of
// Gray levels below vgpr_levels cached in VGPRs (higher ones from L2), tier.
hipError_t launch_walk(int mcols, int vgpr_levels, int tier, const Inst *d_insts, int n_inst,
                       uint64_t total_items, unsigned long long *d_counter, const int32_t *d_k,
                       int waves, hipStream_t stream);

// Whether a (mcols, vgpr_levels) walk variant is compiled in.
bool walk_variant_exists(int mcols, int vgpr_levels);

// Resident walk wavefronts per CU for a variant (occupancy query, >= 1).
int walk_occupancy(int mcols, int vgpr_levels, int tier);

// Per-instance reduction of item results (insts[i].res[0..n_items)), argmin
// rescan (or direct evaluation for tiny n) and float64 rescoring; one
// FinalRes per descriptor.
hipError_t launch_finish(const Inst *d_insts, int n_inst, FinalRes *d_out, hipStream_t stream);

}  // namespace qk

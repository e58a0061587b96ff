// walk_variants.h -- the walk variants' launch and occupancy entry points,
// one pair per translation unit (walk_g12.hip, walk_g12w.hip, walk_g8.hip,
// walk_g6.hip, walk_g5.hip), so that the variants compile in parallel.
#pragma once

#include "kernels.h"

namespace qk {

// Arguments of one walk launch (see launch_walk).
struct WalkLaunch {
    int tier;
    const Inst *insts;
    int n_inst;
    uint64_t total_items;
    unsigned long long *counter;
    const int32_t *k;
    int waves;
    hipStream_t stream;
    const TopkWalk *tk;
};

// Each launch_* returns hipErrorInvalidValue for a column count (or row
// cache) its unit does not build; each occupancy_* returns the resident waves
// per CU of the variant (>= 1).
// 12 VGPR-resident levels, 1, 2 or 4 columns per lane
hipError_t launch_walk_g12(int mcols, const WalkLaunch &w);
int occupancy_walk_g12(int mcols, int tier, int topk_k);
// 12 VGPR-resident levels, 8 or 16 columns per lane
hipError_t launch_walk_g12w(int mcols, const WalkLaunch &w);
int occupancy_walk_g12w(int mcols, int tier, int topk_k);
// 8 VGPR-resident levels, 8 or 16 columns per lane
hipError_t launch_walk_g8(int mcols, const WalkLaunch &w);
int occupancy_walk_g8(int mcols, int tier, int topk_k);
// 16 columns per lane, G = 6: levels 0-5 in VGPRs (lds = false) or levels
// 0-2 and 5 in VGPRs, 3-4 in LDS (lds = true, row cache "4")
hipError_t launch_walk_g6(bool lds, const WalkLaunch &w);
int occupancy_walk_g6(bool lds, int tier, int topk_k);
// 16 columns per lane, G = 5: levels 0-4 in VGPRs (lds = false) or levels
// 0-2 in VGPRs, 3-4 in LDS (lds = true, row cache "3")
hipError_t launch_walk_g5(bool lds, const WalkLaunch &w);
int occupancy_walk_g5(bool lds, int tier, int topk_k);

}  // namespace qk

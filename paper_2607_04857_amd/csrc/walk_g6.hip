// walk_g6.hip -- walk kernel variants: 16 columns per lane, Gray levels 0-5 in VGPRs or levels 0-2 and 5 in VGPRs with 3-4 in LDS.
#include "walk.h"

namespace qk {

hipError_t launch_walk_g6(bool lds, const WalkLaunch &w)
{
    return lds ? launch_walk_g<16, 6, true>(w) : launch_walk_g<16, 6>(w);
}

int occupancy_walk_g6(bool lds, int tier, int topk_k)
{
    return lds ? occupancy_g<16, 6, true>(tier, topk_k) : occupancy_g<16, 6>(tier, topk_k);
}

}  // namespace qk

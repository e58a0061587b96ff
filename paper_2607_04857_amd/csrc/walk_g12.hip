// walk_g12.hip -- walk kernel variants: 12 VGPR-resident levels, 1, 2 or 4 columns per lane.
#include "walk.h"

namespace qk {

hipError_t launch_walk_g12(int mcols, const WalkLaunch &w)
{
    switch (mcols) {
    case 1: return launch_walk_g<1, 12>(w);
    case 2: return launch_walk_g<2, 12>(w);
    case 4: return launch_walk_g<4, 12>(w);
    default: return hipErrorInvalidValue;
    }
}

int occupancy_walk_g12(int mcols, int tier, int topk_k)
{
    switch (mcols) {
    case 1: return occupancy_g<1, 12>(tier, topk_k);
    case 2: return occupancy_g<2, 12>(tier, topk_k);
    case 4: return occupancy_g<4, 12>(tier, topk_k);
    default: return 1;
    }
}

}  // namespace qk

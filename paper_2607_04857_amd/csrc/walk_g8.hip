// walk_g8.hip -- walk kernel variants: 8 VGPR-resident levels, 8 or 16 columns per lane.
#include "walk.h"

namespace qk {

hipError_t launch_walk_g8(int mcols, const WalkLaunch &w)
{
    switch (mcols) {
    case 8: return launch_walk_g<8, 8>(w);
    case 16: return launch_walk_g<16, 8>(w);
    default: return hipErrorInvalidValue;
    }
}

int occupancy_walk_g8(int mcols, int tier, int topk_k)
{
    switch (mcols) {
    case 8: return occupancy_g<8, 8>(tier, topk_k);
    case 16: return occupancy_g<16, 8>(tier, topk_k);
    default: return 1;
    }
}

}  // namespace qk

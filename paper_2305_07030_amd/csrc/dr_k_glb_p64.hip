// Instantiates the global-placement DR kernel k_dr_glb<P64, BLOCK, C>, one
// workgroup per problem, and its group form k_dr_glb<P64, BLOCK, C, true>
// (the tail hand-off's cooperative launch).
#include "dr_device.h"

namespace drk {
int launch_glb_p64(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st)
{
    return launch_glb_all<P64>(a, pl, st);
}

int launch_group_p64(const SolveArgs &a, const LaunchPlan &pl, int grid, hipStream_t st)
{
    if (pl.block == 1024) return launch_group<P64, 1024, 1>(a, pl, grid, st);
    if (pl.block == 512) return launch_group<P64, 512, 2>(a, pl, grid, st);
    return -1001;
}

int group_capacity_p64(int block, int lds_bytes, int *blocks_per_cu)
{
    if (block == 1024) return group_occupancy<P64, 1024, 1>(lds_bytes, blocks_per_cu);
    if (block == 512) return group_occupancy<P64, 512, 2>(lds_bytes, blocks_per_cu);
    return -1001;
}
} // namespace drk

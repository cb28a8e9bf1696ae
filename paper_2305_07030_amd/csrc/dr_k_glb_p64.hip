// Instantiates the global-placement DR kernel k_dr_glb<P64, BLOCK, C>.
#include "dr_device.h"

namespace drk {
int launch_glb_p64(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st)
{
    return launch_glb_all<P64>(a, pl, st);
}
} // namespace drk

// Instantiates the register/LDS-resident DR kernel k_dr_reg<P64, 512, NPT, CH>.
#include "dr_device.h"

namespace drk {
int launch_reg_p64_512(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st)
{
    return launch_reg<P64, 512>(a, pl, st);
}
} // namespace drk

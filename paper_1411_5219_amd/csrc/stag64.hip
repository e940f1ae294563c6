// FP64-storage instantiations of the even-odd staggered hop kernels.
#include "staggered_impl.h"

namespace lqcd {

hipError_t launch_stag_64(int recon, int red, bool lnt, const DslashLaunch& L, dim3 grid, dim3 block, hipStream_t s)
{
    if (recon == 18) return launch_stag_red<64, 18>(red, lnt, L, grid, block, s);
    if (recon == 12) return launch_stag_red<64, 12>(red, lnt, L, grid, block, s);
    return hipErrorInvalidValue;
}

}  // namespace lqcd

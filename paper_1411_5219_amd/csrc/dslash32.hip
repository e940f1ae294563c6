// FP32-storage instantiations of the even-odd Dslash kernels.
#include "dslash_impl.h"

namespace lqcd {

hipError_t launch_dslash_32(int recon, int nr, bool lnt, bool dag, int red, const DslashLaunch& L, dim3 grid, dim3 block,
                               hipStream_t s)
{
    if (recon == 18) return launch_tile<32, 18>(nr, lnt, dag, red, L, grid, block, s);
    if (recon == 12) return launch_tile<32, 12>(nr, lnt, dag, red, L, grid, block, s);
    return hipErrorInvalidValue;
}

}  // namespace lqcd

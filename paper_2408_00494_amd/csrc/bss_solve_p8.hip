// bss_solve_p8.hip -- solve kernel variants with 8 particles per lane.
#include "bss_solve.h"

namespace bss {

hipError_t launch_solve_p8(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                          bool shield, bool split, bool resample, bool con, size_t lds,
                          const double* x0_base, const double* Sigma0_base, int extra_shift,
                          uint32_t* queue, hipStream_t stream)
{
    return launch_solve_p<8>(inst, blocks, nblocks, shield, split, resample, con, lds, x0_base,
                             Sigma0_base, extra_shift, queue, stream);
}

}  // namespace bss

// bss_solve_pm.hip -- solve kernel variants that take the particles per lane from each instance
// (batches whose members run different P in one launch).
#include "bss_solve.h"

namespace bss {

hipError_t launch_solve_pm(const InstanceDesc* inst, const BlockDesc* blocks, int nblocks,
                           bool shield, bool split, bool resample, bool con, size_t lds,
                           const double* x0_base, const double* Sigma0_base, int extra_shift,
                           uint32_t* queue, hipStream_t stream)
{
    if (shield || resample || con) return hipErrorInvalidValue;
    if (split)
        return launch_variant<0, false, true, false, false>(inst, blocks, nblocks, lds, x0_base,
                                                            Sigma0_base, extra_shift, queue,
                                                            stream);
    return launch_variant<0, false, false, false, false>(inst, blocks, nblocks, lds, x0_base,
                                                         Sigma0_base, extra_shift, queue, stream);
}

}  // namespace bss

// Batched ensembles under draw specification v2 (Philox4x32 with seven
// rounds): the persistent kernel's instantiations for D1Q2, D1Q3 and D2Q5.
#include "batch_kernel.h"

namespace ilg {

hipError_t launch_batch_p7(int q, int count_bytes, int shape, const BatchArgs &a,
                           hipStream_t stream)
{
    if (q == 2 && count_bytes == 2)
        return launch_qt<2, uint16_t, 7, false>(shape, a, stream);
    if (q == 2 && count_bytes == 4)
        return launch_qt<2, uint32_t, 7, false>(shape, a, stream);
    if (q == 3 && count_bytes == 2)
        return launch_qt<3, uint16_t, 7, false>(shape, a, stream);
    if (q == 3 && count_bytes == 4)
        return launch_qt<3, uint32_t, 7, false>(shape, a, stream);
    if (q == 5 && count_bytes == 2)
        return launch_qt<5, uint16_t, 7, false>(shape, a, stream);
    if (q == 5 && count_bytes == 4)
        return launch_qt<5, uint32_t, 7, false>(shape, a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ilg

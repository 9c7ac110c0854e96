// Batched D1Q2 ensembles under draw specification v3 (the exchange form,
// with ten- or seven-round draws): the persistent kernel's instantiations.
#include "batch_kernel.h"

namespace ilg {

hipError_t launch_batch_ex(int q, int count_bytes, int shape, const BatchArgs &a,
                           hipStream_t stream)
{
    if (q != 2)
        return hipErrorInvalidValue;
    if (a.rounds == 7)
        return count_bytes == 2 ? launch_qt<2, uint16_t, 7, true>(shape, a, stream)
                                : launch_qt<2, uint32_t, 7, true>(shape, a, stream);
    if (a.rounds == 10)
        return count_bytes == 2 ? launch_qt<2, uint16_t, 10, true>(shape, a, stream)
                                : launch_qt<2, uint32_t, 10, true>(shape, a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ilg

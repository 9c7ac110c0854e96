// Batched ensembles: launch entry points and the ten-round instantiations of
// the persistent kernel (batch_kernel.h).
#include "batch_kernel.h"

namespace ilg {

namespace {

__global__ void batch_reset_kernel(uint32_t *queue)
{
    if (threadIdx.x == 0)
        *queue = 0u;
}

}  // namespace

int batch_shape_count()
{
    return (int)(sizeof(kShapes) / sizeof(kShapes[0]));
}

void batch_shape(int shape, int q, int *block, int *wg_per_cu)
{
    *block = kShapes[shape].block;
    *wg_per_cu = q == 2 ? kShapes[shape].wg_per_cu_q2 : kShapes[shape].wg_per_cu_q3;
}

hipError_t launch_batch_reset(uint32_t *queue, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, stream, queue);
    return hipGetLastError();
}

hipError_t launch_batch(int q, int count_bytes, int shape, const BatchArgs &a, hipStream_t stream)
{
    if (shape < 0 || shape >= batch_shape_count())
        return hipErrorInvalidValue;
    if (a.exchange)
        return launch_batch_ex(q, count_bytes, shape, a, stream);
    if (a.rounds == 7)
        return launch_batch_p7(q, count_bytes, shape, a, stream);
    if (a.rounds != 10)
        return hipErrorInvalidValue;
    if (q == 2 && count_bytes == 2)
        return launch_qt<2, uint16_t, 10, false>(shape, a, stream);
    if (q == 2 && count_bytes == 4)
        return launch_qt<2, uint32_t, 10, false>(shape, a, stream);
    if (q == 3 && count_bytes == 2)
        return launch_qt<3, uint16_t, 10, false>(shape, a, stream);
    if (q == 3 && count_bytes == 4)
        return launch_qt<3, uint32_t, 10, false>(shape, a, stream);
    if (q == 5 && count_bytes == 2)
        return launch_qt<5, uint16_t, 10, false>(shape, a, stream);
    if (q == 5 && count_bytes == 4)
        return launch_qt<5, uint32_t, 10, false>(shape, a, stream);
    return hipErrorInvalidValue;
}

}  // namespace ilg

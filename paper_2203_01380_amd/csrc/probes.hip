// Measurement probes for the roofline of the fused step (not part of the
// method): each isolates one of the two costs the step kernel combines, with
// the step kernel's own launch shape (1024-thread workgroups, two per CU, a
// persistent grid whose workgroups of one XCD cover one contiguous eighth of
// the lattice, one node per thread).
//
//  * Streaming only: the memory pattern of the D1Q3 / D1Q2 uint16 step (the
//    rows of Eq. ilgeq's left side: every count read once, the -1 and +1
//    populations stored one node off, periodic), with no flip and no
//    collision.  Its rate is the achievable HBM rate of the step's traffic.
//  * Draws only: for every node, the Philox4x32 blocks (x, t, realization,
//    b), b < blocks, that the step draws (two per D1Q3 node), folded by xor
//    into one word per node so that none can be dropped.  Its rate bounds the
//    step from the draw side.
#include "ilg_internal.h"
#include "philox.h"

namespace ilg {

namespace {

constexpr int kNumXcd = 8;
constexpr int kBlock = 1024;
constexpr int kWgPerCu = 2;

// Tiles [first, end) of this workgroup, stride `stride` (as the step kernel).
__device__ __forceinline__ void xcd_tiles(uint32_t ntiles, uint32_t &first, uint32_t &end,
                                          uint32_t &stride)
{
    if (gridDim.x % kNumXcd == 0) {
        const uint32_t xcd = blockIdx.x % kNumXcd;
        first = (uint32_t)((uint64_t)ntiles * xcd / kNumXcd) + blockIdx.x / kNumXcd;
        end = (uint32_t)((uint64_t)ntiles * (xcd + 1) / kNumXcd);
        stride = gridDim.x / kNumXcd;
    } else {
        first = blockIdx.x;
        end = ntiles;
        stride = gridDim.x;
    }
}

template <int Q>
__global__ __launch_bounds__(kBlock) void stream_probe_kernel(const uint16_t *in, uint16_t *out,
                                                              uint64_t pitch, uint32_t length)
{
    uint32_t first, end, stride;
    xcd_tiles((length + kBlock - 1) / kBlock, first, end, stride);
    for (uint32_t tile = first; tile < end; tile += stride) {
        const uint32_t x = tile * kBlock + threadIdx.x;
        if (x >= length)
            continue;
        const uint32_t xm = (x == 0) ? length - 1 : x - 1;
        const uint32_t xp = (x + 1 == length) ? 0 : x + 1;
        const uint16_t a = in[x];
        const uint16_t c = in[(uint64_t)(Q - 1) * pitch + x];
        out[xm] = a;
        out[(uint64_t)(Q - 1) * pitch + xp] = c;
        if constexpr (Q == 3)
            out[pitch + x] = in[pitch + x];
    }
}

template <int NR>
__global__ __launch_bounds__(kBlock) void philox_probe_kernel(uint32_t *out, uint32_t length,
                                                              uint32_t blocks, uint32_t t,
                                                              uint32_t r, uint32_t k0,
                                                              uint32_t k1)
{
    uint32_t first, end, stride;
    xcd_tiles((length + kBlock - 1) / kBlock, first, end, stride);
    for (uint32_t tile = first; tile < end; tile += stride) {
        const uint32_t x = tile * kBlock + threadIdx.x;
        if (x >= length)
            continue;
        uint32_t acc = 0;
        for (uint32_t b = 0; b < blocks; ++b) {
            const uint4 o = philox4x32<NR>(x, t, r, b, k0, k1);
            acc ^= xor3(o.x, o.y, o.z) ^ o.w;
        }
        out[x] = acc;
    }
}

uint32_t probe_grid(uint32_t length)
{
    const uint32_t ntiles = (length + kBlock - 1) / kBlock;
    uint32_t grid = (uint32_t)device_cu_count() * kWgPerCu;
    if (ntiles < grid)
        grid = ntiles;
    if (grid >= (uint32_t)kNumXcd)
        grid -= grid % kNumXcd;
    return grid == 0 ? 1 : grid;
}

}  // namespace

}  // namespace ilg

extern "C" {

int ilg_probe_stream(uint32_t q, uint64_t length, const void *in_dev, void *out_dev, void *stream)
{
    if ((q != 2 && q != 3) || length < 1 || length >= (uint64_t(1) << 31) || !in_dev || !out_dev) {
        ilg::set_last_error("need q = 2 or 3, 1 <= length < 2^31 and two device buffers");
        return ILG_E_INVALID;
    }
    const uint64_t pitch = (length + 63) / 64 * 64;
    const uint32_t L = (uint32_t)length;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const auto *in = static_cast<const uint16_t *>(in_dev);
    auto *out = static_cast<uint16_t *>(out_dev);
    if (q == 3)
        hipLaunchKernelGGL(ilg::stream_probe_kernel<3>, dim3(ilg::probe_grid(L)),
                           dim3(ilg::kBlock), 0, s, in, out, pitch, L);
    else
        hipLaunchKernelGGL(ilg::stream_probe_kernel<2>, dim3(ilg::probe_grid(L)),
                           dim3(ilg::kBlock), 0, s, in, out, pitch, L);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        ilg::set_last_error(std::string("stream probe launch: ") + hipGetErrorString(e));
        return ILG_E_DEVICE;
    }
    return ILG_OK;
}

int ilg_probe_philox(uint64_t length, uint32_t blocks, uint32_t rounds, uint32_t t, uint64_t seed,
                     void *out_dev, void *stream)
{
    if (length < 1 || length >= (uint64_t(1) << 31) || blocks < 1 || blocks > 64 ||
        (rounds != 10 && rounds != 7) || !out_dev) {
        ilg::set_last_error("need 1 <= length < 2^31, 1 <= blocks <= 64, rounds 10 or 7 and an "
                            "output buffer");
        return ILG_E_INVALID;
    }
    const uint32_t L = (uint32_t)length;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    auto *out = static_cast<uint32_t *>(out_dev);
    const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
    if (rounds == 10)
        hipLaunchKernelGGL(ilg::philox_probe_kernel<10>, dim3(ilg::probe_grid(L)),
                           dim3(ilg::kBlock), 0, s, out, L, blocks, t, 0u, k0, k1);
    else
        hipLaunchKernelGGL(ilg::philox_probe_kernel<7>, dim3(ilg::probe_grid(L)),
                           dim3(ilg::kBlock), 0, s, out, L, blocks, t, 0u, k0, k1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        ilg::set_last_error(std::string("Philox probe launch: ") + hipGetErrorString(e));
        return ILG_E_DEVICE;
    }
    return ILG_OK;
}

}  // extern "C"

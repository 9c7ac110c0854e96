// ilg_step_noalloc: the steps of ilg_step for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  The caller owns the two state buffers;
// everything else the step kernel needs, the fixed-point table set it stages
// into LDS and the sticky error word, lives in `scratch`, a fixed array of
// this library on each device.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// its device address is taken once per device with hipGetSymbolAddress (with
// that device current) and only that address is used afterwards.
#include <cfenv>
#include <cstring>
#include <mutex>
#include <string>

#include "ilg.h"
#include "ilg_internal.h"

namespace {

// Table set, then the error word on its own 256-byte line.
constexpr size_t kErrOffset = (ilg::kTableSetBytes + 255) / 256 * 256;
constexpr size_t kScratchBytes = kErrOffset + 256;
static_assert(kScratchBytes == ILG_NOALLOC_SCRATCH_BYTES, "scratch size stated in ilg.h");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void *g_scratch[kMaxDevices];
hipError_t g_symbol_err[kMaxDevices];

// Host copy of the table set of the last call on this thread.
thread_local unsigned char t_tables[ilg::kTableSetBytes];

int fail(int code, const std::string &msg)
{
    ilg::set_last_error(msg);
    return code;
}

}  // namespace

extern "C" int ilg_step_noalloc(const ilg_config *cfg, void *buf0, void *buf1, uint64_t nsteps,
                                void *stream, uint32_t sync)
{
    ilg::Fixed fx;
    int rc = ilg::check_config(cfg, &fx);
    if (rc != ILG_OK)
        return rc;
    if (!buf0 || !buf1 || buf0 == buf1)
        return fail(ILG_E_INVALID, "ilg_step_noalloc: need two distinct device buffers");
    if (cfg->t0 + nsteps > (uint64_t(1) << 32))
        return fail(ILG_E_RANGE, "ilg_step_noalloc: step index would pass 2^32 - 1");
    // The scratch array holds only the table set and the error word (the
    // static_assert above): its use does not grow with the lattice, whose
    // state the caller owns and whose size check_config bounds.
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(ILG_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(ILG_E_DEVICE, "ilg_step_noalloc: device index beyond the supported 64");
    std::call_once(g_once[dev], [dev]() {
        g_symbol_err[dev] = hipGetSymbolAddress(&g_scratch[dev], HIP_SYMBOL(scratch));
    });
    if (g_symbol_err[dev] != hipSuccess || !g_scratch[dev])
        return fail(ILG_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(g_symbol_err[dev]));
    unsigned char *sp = static_cast<unsigned char *>(g_scratch[dev]);
    uint32_t *err = reinterpret_cast<uint32_t *>(sp + kErrOffset);
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    // This call's table set, copied into the scratch array on the stream
    // (every call: the array keeps only the last call's tables).
    ilg::build_table_set(fx.p, fx.p_rest, t_tables);
    e = hipMemcpyAsync(sp, t_tables, ilg::kTableSetBytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return fail(ILG_E_DEVICE, std::string("table copy: ") + hipGetErrorString(e));

    const uint64_t nodes = cfg->length * (cfg->q == 5 ? (uint64_t)cfg->height : 1u);
    ilg::StepArgs a;
    a.pitch = (nodes + 63) / 64 * 64;
    a.length = (uint32_t)nodes;
    a.width = (uint32_t)cfg->length;
    a.height = cfg->q == 5 ? cfg->height : 1u;
    a.realization = cfg->realization;
    a.key0 = (uint32_t)(cfg->seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(cfg->seed >> 32);
    a.flip = (uint32_t)fx.flip;
    a.p_zero = fx.p == 0 ? 1u : 0u;
    a.rounds = (uint32_t)fx.rounds;
    a.exchange = (uint32_t)fx.exchange;
    a.tables = sp;
    a.err = err;
    void *buf[2] = {buf0, buf1};
    for (uint64_t k = 0; k < nsteps; ++k) {
        a.in = buf[k & 1];
        a.out = buf[(k & 1) ^ 1];
        a.t = (uint32_t)(cfg->t0 + k);
        e = ilg::launch_step((int)cfg->q, (int)cfg->count_bytes, a, s);
        if (e != hipSuccess)
            return fail(ILG_E_DEVICE, std::string("step launch: ") + hipGetErrorString(e));
    }
    if (!sync)
        return ILG_OK;
    uint32_t word = 0;
    e = hipMemcpyAsync(&word, err, sizeof(word), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(ILG_E_DEVICE, std::string("error word: ") + hipGetErrorString(e));
    if (word & 1u) {
        // reported once: the word starts again from zero
        e = hipMemsetAsync(err, 0, sizeof(uint32_t), s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return fail(ILG_E_DEVICE, std::string("error word reset: ") + hipGetErrorString(e));
        return fail(ILG_E_OVERFLOW, "a post-collision count exceeded the count type");
    }
    return ILG_OK;
}

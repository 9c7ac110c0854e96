// Host runtime behind the C ABI of include/ilg.h: configuration checks, the
// fixed-point parameters, device buffers and tables, step launches and the
// syncing query calls.
#include <cfenv>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ilg.h"
#include "ilg_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(ILG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define ILG_HIP(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess)                          \
            return hip_fail(e_, #call);                \
    } while (0)

uint64_t pitch_of(uint64_t length)
{
    return (length + 63) / 64 * 64;
}

// Nodes of a configuration: L in 1D, Lx Ly for D2Q5 (node x + Lx y).
uint64_t nodes_of(const ilg_config *cfg)
{
    return cfg->length * (cfg->q == 5 ? (uint64_t)cfg->height : 1u);
}

}  // namespace

struct ilg_handle {
    ilg_config cfg;
    ilg::Fixed fx;
    hipStream_t stream = nullptr;
    void *buf[2] = {nullptr, nullptr};
    bool owns_state = false;
    int cur = 0;
    uint64_t pitch = 0, bytes = 0;
    void *tables = nullptr;   // device table set
    uint32_t *err = nullptr;  // device sticky error word
    void *diag_partials = nullptr;
    void *diag_result = nullptr;
    int64_t *mom = nullptr;   // 3 * L int64 per-node moments (lazy)
    uint64_t t = 0;           // absolute index of the next step
};

namespace ilg {

int device_cu_count()
{
    static int cached = 0;
    if (cached > 0)
        return cached;
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
        n = 256;
    cached = n;
    return n;
}

void set_last_error(const std::string &msg)
{
    g_last_error = msg;
}

// Validates cfg and derives the fixed-point parameters (Over-relaxation
// section: omega* in [0, 1] after the flip; Eq. omegaj: omega^j = 2 - omega*).
int check_config(const ilg_config *cfg, Fixed *fx)
{
    if (!cfg)
        return fail(ILG_E_INVALID, "null config");
    if (cfg->abi_version != ILG_ABI_VERSION)
        return fail(ILG_E_INVALID, "abi_version mismatch");
    if (cfg->q != 2 && cfg->q != 3 && cfg->q != 5)
        return fail(ILG_E_INVALID, "q must be 2, 3 or 5");
    if (cfg->count_bytes != 2 && cfg->count_bytes != 4)
        return fail(ILG_E_INVALID, "count_bytes must be 2 or 4");
    if (cfg->length < 1 || cfg->length >= (uint64_t(1) << 31))
        return fail(ILG_E_INVALID, "length must be in [1, 2^31)");
    if (cfg->q == 5 ? cfg->height < 1 : cfg->height != 0)
        return fail(ILG_E_INVALID, "height must be >= 1 for q = 5 and 0 otherwise");
    if (nodes_of(cfg) >= (uint64_t(1) << 31))
        return fail(ILG_E_INVALID, "the node count must be below 2^31");
    if ((cfg->flags & ~(ILG_FLIP_MASK | ILG_DRAWS_PHILOX7 | ILG_DRAWS_EXCHANGE)) != 0)
        return fail(ILG_E_INVALID, "reserved flag bits set");
    if ((cfg->flags & ILG_DRAWS_EXCHANGE) && cfg->q != 2)
        return fail(ILG_E_INVALID, "the exchange form is defined for q = 2");
    if (!(cfg->omega > 0.0 && cfg->omega <= 2.0))
        return fail(ILG_E_INVALID, "omega must lie in (0, 2]");
    if (cfg->t0 > 0xFFFFFFFFull)
        return fail(ILG_E_RANGE, "t0 must be below 2^32");
    double theta = cfg->theta == 0.0 ? 1.0 / 3.0 : cfg->theta;
    if (cfg->q == 3 && !(theta > 0.0 && theta < 1.0))
        return fail(ILG_E_INVALID, "theta must lie in (0, 1)");
    if (cfg->q == 5 && !(theta > 0.0 && theta < 0.5))
        return fail(ILG_E_INVALID, "D2Q5 theta must lie in (0, 1/2)");
    bool flip;
    switch (cfg->flags & ILG_FLIP_MASK) {
    case ILG_FLIP_AUTO:
        flip = cfg->omega > 1.0;
        break;
    case ILG_FLIP_OFF:
        if (cfg->omega > 1.0)
            return fail(ILG_E_INVALID, "omega > 1 needs the flip");
        flip = false;
        break;
    case ILG_FLIP_ON:
        if (cfg->omega < 1.0)
            return fail(ILG_E_INVALID, "a forced flip needs omega >= 1");
        flip = true;
        break;
    default:
        return fail(ILG_E_INVALID, "bad flip mode");
    }
    const double omega_star = flip ? 2.0 - cfg->omega : cfg->omega;
    // round half to even in IEEE double (default rounding mode)
    const int saved = std::fegetround();
    std::fesetround(FE_TONEAREST);
    const double two32 = 4294967296.0;
    fx->flip = flip ? 1 : 0;
    fx->rounds = (cfg->flags & ILG_DRAWS_PHILOX7) ? 7 : 10;
    fx->omega_star = omega_star;
    fx->exchange = (cfg->flags & ILG_DRAWS_EXCHANGE) ? 1 : 0;
    // exchange form: the crossing probability omega* / 2 (omega* 2^31 is exact)
    fx->p = (uint64_t)std::nearbyint(omega_star * (fx->exchange ? two32 / 2.0 : two32));
    fx->p_half = uint64_t(1) << 31;
    fx->p_rest = cfg->q == 3   ? (uint64_t)std::nearbyint((1.0 - theta) * two32)
                 : cfg->q == 5 ? (uint64_t)std::nearbyint((1.0 - 2.0 * theta) * two32)
                               : 0;
    std::fesetround(saved);
    return ILG_OK;
}

StepArgs step_args(const ilg_handle *h)
{
    StepArgs a;
    a.in = h->buf[h->cur];
    a.out = h->buf[h->cur ^ 1];
    a.pitch = h->pitch;
    a.length = (uint32_t)nodes_of(&h->cfg);
    a.width = (uint32_t)h->cfg.length;
    a.height = h->cfg.q == 5 ? h->cfg.height : 1u;
    a.t = (uint32_t)h->t;
    a.realization = h->cfg.realization;
    a.key0 = (uint32_t)(h->cfg.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(h->cfg.seed >> 32);
    a.flip = (uint32_t)h->fx.flip;
    a.p_zero = h->fx.p == 0 ? 1u : 0u;
    a.rounds = (uint32_t)h->fx.rounds;
    a.exchange = (uint32_t)h->fx.exchange;
    a.tables = h->tables;
    a.err = h->err;
    return a;
}

}  // namespace ilg

namespace {

int alloc_common(ilg_handle *h)
{
    std::vector<unsigned char> set(ilg::kTableSetBytes);
    ilg::build_table_set(h->fx.p, h->fx.p_rest, set.data());
    ILG_HIP(hipMalloc(&h->tables, ilg::kTableSetBytes));
    ILG_HIP(hipMemcpyAsync(h->tables, set.data(), set.size(), hipMemcpyHostToDevice, h->stream));
    ILG_HIP(hipMalloc((void **)&h->err, sizeof(uint32_t)));
    ILG_HIP(hipMemsetAsync(h->err, 0, sizeof(uint32_t), h->stream));
    ILG_HIP(hipMalloc(&h->diag_partials, ilg::diag_partials_bytes()));
    ILG_HIP(hipMalloc(&h->diag_result, sizeof(ilg::DiagResult)));
    ILG_HIP(hipStreamSynchronize(h->stream));
    return ILG_OK;
}

void release(ilg_handle *h)
{
    if (h->owns_state) {
        (void)hipFree(h->buf[0]);
        (void)hipFree(h->buf[1]);
    }
    (void)hipFree(h->tables);
    (void)hipFree(h->err);
    (void)hipFree(h->diag_partials);
    (void)hipFree(h->diag_result);
    (void)hipFree(h->mom);
    delete h;
}

int check_sticky(ilg_handle *h)
{
    uint32_t err = 0;
    ILG_HIP(hipMemcpyAsync(&err, h->err, sizeof(err), hipMemcpyDeviceToHost, h->stream));
    ILG_HIP(hipStreamSynchronize(h->stream));
    if (err & 1u)
        return fail(ILG_E_OVERFLOW, "a post-collision count exceeded the count type");
    return ILG_OK;
}

int copy_state_in(ilg_handle *h, const void *host)
{
    const size_t cb = h->cfg.count_bytes;
    const size_t n = nodes_of(&h->cfg);
    ILG_HIP(hipMemcpy2DAsync(h->buf[h->cur], h->pitch * cb, host, n * cb, n * cb, h->cfg.q,
                             hipMemcpyHostToDevice, h->stream));
    ILG_HIP(hipStreamSynchronize(h->stream));
    return ILG_OK;
}

}  // namespace

extern "C" {

const char *ilg_last_error(void)
{
    return g_last_error.c_str();
}

int ilg_fixed_point(const ilg_config *cfg, ilg_fixed *out)
{
    if (!out)
        return fail(ILG_E_INVALID, "null output");
    ilg::Fixed fx;
    int rc = ilg::check_config(cfg, &fx);
    if (rc != ILG_OK)
        return rc;
    out->flip = (uint32_t)fx.flip;
    out->q = cfg->q;
    out->p = fx.p;
    out->p_half = fx.p_half;
    out->p_rest = fx.p_rest;
    out->omega_star = fx.omega_star;
    return ILG_OK;
}

int ilg_binomial_table(uint64_t p, uint32_t *out)
{
    if (!out || p == 0 || p > (uint64_t(1) << 32))
        return fail(ILG_E_INVALID, "p must lie in (0, 2^32]");
    ilg::build_binomial_table(p, out);
    return ILG_OK;
}

uint64_t ilg_state_pitch(const ilg_config *cfg)
{
    return cfg ? pitch_of(nodes_of(cfg)) : 0;
}

uint64_t ilg_state_bytes(const ilg_config *cfg)
{
    return cfg ? pitch_of(nodes_of(cfg)) * cfg->q * cfg->count_bytes : 0;
}

static int create_common(const ilg_config *cfg, void *stream, ilg_handle **out, ilg_handle **hp)
{
    if (!out)
        return fail(ILG_E_INVALID, "null output handle");
    *out = nullptr;
    ilg::Fixed fx;
    int rc = ilg::check_config(cfg, &fx);
    if (rc != ILG_OK)
        return rc;
    ilg_handle *h = new (std::nothrow) ilg_handle;
    if (!h)
        return fail(ILG_E_NOMEM, "host allocation failed");
    h->cfg = *cfg;
    if (h->cfg.theta == 0.0)
        h->cfg.theta = 1.0 / 3.0;
    h->fx = fx;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    h->pitch = pitch_of(nodes_of(cfg));
    h->bytes = h->pitch * cfg->q * cfg->count_bytes;
    h->t = cfg->t0;
    *hp = h;
    return ILG_OK;
}

int ilg_create(const ilg_config *cfg, const void *init_host, void *stream, ilg_handle **out)
{
    ilg_handle *h = nullptr;
    int rc = create_common(cfg, stream, out, &h);
    if (rc != ILG_OK)
        return rc;
    h->owns_state = true;
    hipError_t e1 = hipMalloc(&h->buf[0], h->bytes);
    hipError_t e2 = hipMalloc(&h->buf[1], h->bytes);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        release(h);
        return fail(ILG_E_NOMEM, "device allocation of the state failed");
    }
    rc = alloc_common(h);
    if (rc == ILG_OK && init_host) {
        rc = copy_state_in(h, init_host);
    } else if (rc == ILG_OK) {
        // no initial state: zero counts (for a device-side initialisation)
        if (hipMemsetAsync(h->buf[0], 0, h->bytes, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            rc = fail(ILG_E_DEVICE, "zeroing the state failed");
    }
    if (rc != ILG_OK) {
        std::string msg = g_last_error;
        release(h);
        return fail(rc, msg);
    }
    *out = h;
    return ILG_OK;
}

int ilg_create_on(const ilg_config *cfg, void *buf0, void *buf1, void *stream, ilg_handle **out)
{
    ilg_handle *h = nullptr;
    int rc = create_common(cfg, stream, out, &h);
    if (rc != ILG_OK)
        return rc;
    if (!buf0 || !buf1 || buf0 == buf1) {
        delete h;
        return fail(ILG_E_INVALID, "need two distinct device buffers");
    }
    h->owns_state = false;
    h->buf[0] = buf0;
    h->buf[1] = buf1;
    rc = alloc_common(h);
    if (rc != ILG_OK) {
        std::string msg = g_last_error;
        release(h);
        return fail(rc, msg);
    }
    *out = h;
    return ILG_OK;
}

void *ilg_state_device(const ilg_handle *h)
{
    return h ? h->buf[h->cur] : nullptr;
}

uint64_t ilg_current_step(const ilg_handle *h)
{
    return h ? h->t : 0;
}

int ilg_step(ilg_handle *h, uint64_t nsteps)
{
    if (!h)
        return fail(ILG_E_INVALID, "null handle");
    if (h->t + nsteps > (uint64_t(1) << 32))
        return fail(ILG_E_RANGE, "step index would pass 2^32 - 1");
    for (uint64_t s = 0; s < nsteps; ++s) {
        ilg::StepArgs a = ilg::step_args(h);
        hipError_t e = ilg::launch_step((int)h->cfg.q, (int)h->cfg.count_bytes, a, h->stream);
        if (e != hipSuccess)
            return hip_fail(e, "step launch");
        h->cur ^= 1;
        h->t += 1;
    }
    return ILG_OK;
}

int ilg_get_state(ilg_handle *h, void *host_out)
{
    if (!h || !host_out)
        return fail(ILG_E_INVALID, "null argument");
    const size_t cb = h->cfg.count_bytes;
    const size_t n = nodes_of(&h->cfg);
    ILG_HIP(hipMemcpy2DAsync(host_out, n * cb, h->buf[h->cur], h->pitch * cb, n * cb, h->cfg.q,
                             hipMemcpyDeviceToHost, h->stream));
    return check_sticky(h);
}

int ilg_set_state(ilg_handle *h, const void *host_in, uint64_t t)
{
    if (!h || !host_in)
        return fail(ILG_E_INVALID, "null argument");
    if (t > 0xFFFFFFFFull)
        return fail(ILG_E_RANGE, "t must be below 2^32");
    int rc = copy_state_in(h, host_in);
    if (rc != ILG_OK)
        return rc;
    ILG_HIP(hipMemsetAsync(h->err, 0, sizeof(uint32_t), h->stream));
    ILG_HIP(hipStreamSynchronize(h->stream));
    h->t = t;
    return ILG_OK;
}

int ilg_init_poisson_sine(ilg_handle *h, double nave, double amp, uint64_t init_seed)
{
    if (!h)
        return fail(ILG_E_INVALID, "null handle");
    if (!std::isfinite(nave) || !std::isfinite(amp) || nave < 0.0 || nave > 1.0e6 ||
        std::fabs(amp) > nave)
        return fail(ILG_E_INVALID, "need 0 <= nave <= 1e6 and |amp| <= nave");
    const double theta = h->cfg.theta == 0.0 ? 1.0 / 3.0 : h->cfg.theta;
    ilg::InitArgs a;
    a.out = h->buf[h->cur ^ 1];
    a.pitch = h->pitch;
    a.length = (uint32_t)nodes_of(&h->cfg);
    a.width = (uint32_t)h->cfg.length;
    a.q = h->cfg.q;
    a.realization = h->cfg.realization;
    a.key0 = (uint32_t)(init_seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(init_seed >> 32);
    for (int i = 0; i < 5; ++i)
        a.w[i] = 0.0;
    if (h->cfg.q == 2) {
        a.w[0] = 0.5;
        a.w[1] = 0.5;
    } else if (h->cfg.q == 3) {
        a.w[0] = theta * 0.5;
        a.w[1] = 1.0 - theta;
        a.w[2] = theta * 0.5;
    } else {
        a.w[0] = theta * 0.5;
        a.w[1] = theta * 0.5;
        a.w[2] = 1.0 - 2.0 * theta;
        a.w[3] = theta * 0.5;
        a.w[4] = theta * 0.5;
    }
    a.nave = nave;
    a.amp = amp;
    a.err = h->err;
    ILG_HIP(hipMemsetAsync(h->err, 0, sizeof(uint32_t), h->stream));
    hipError_t e = ilg::launch_init((int)h->cfg.count_bytes, a, h->stream);
    if (e != hipSuccess)
        return hip_fail(e, "init launch");
    uint32_t err = 0;
    ILG_HIP(hipMemcpyAsync(&err, h->err, sizeof(err), hipMemcpyDeviceToHost, h->stream));
    ILG_HIP(hipStreamSynchronize(h->stream));
    if (err & 1u) {
        ILG_HIP(hipMemsetAsync(h->err, 0, sizeof(uint32_t), h->stream));
        ILG_HIP(hipStreamSynchronize(h->stream));
        return fail(ILG_E_OVERFLOW, "an initial count exceeds the count type (state unchanged)");
    }
    h->cur ^= 1;
    return ILG_OK;
}

static int run_diag(ilg_handle *h, bool moments, uint32_t nk, ilg::DiagResult *res)
{
    ilg::DiagArgs a;
    a.state = h->buf[h->cur];
    const uint64_t n = nodes_of(&h->cfg);
    a.pitch = h->pitch;
    a.length = (uint32_t)n;
    a.width = (uint32_t)h->cfg.length;
    a.q = h->cfg.q;
    a.count_bytes = h->cfg.count_bytes;
    a.nk = nk;
    a.rho = a.j = a.e = nullptr;
    if (moments) {
        if (!h->mom)
            ILG_HIP(hipMalloc((void **)&h->mom, 3 * n * sizeof(int64_t)));
        a.rho = h->mom;
        a.j = h->mom + n;
        a.e = h->mom + 2 * n;
    }
    a.partials = h->diag_partials;
    a.result = h->diag_result;
    hipError_t e = ilg::launch_diag(a, h->stream);
    if (e != hipSuccess)
        return hip_fail(e, "diagnostics launch");
    ILG_HIP(hipMemcpyAsync(res, h->diag_result, sizeof(*res), hipMemcpyDeviceToHost, h->stream));
    return ILG_OK;
}

int ilg_moments(ilg_handle *h, int64_t *rho, int64_t *j, int64_t *e, uint32_t nk,
                ilg_summary *out)
{
    if (!h || !out)
        return fail(ILG_E_INVALID, "null argument");
    if (nk > ILG_MAX_K)
        return fail(ILG_E_INVALID, "nk exceeds ILG_MAX_K");
    const bool moments = rho || j || e;
    ilg::DiagResult res;
    int rc = run_diag(h, moments, nk, &res);
    if (rc != ILG_OK)
        return rc;
    const uint64_t L = nodes_of(&h->cfg);
    if (rho)
        ILG_HIP(hipMemcpyAsync(rho, h->mom, L * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
    if (j)
        ILG_HIP(hipMemcpyAsync(j, h->mom + L, L * sizeof(int64_t), hipMemcpyDeviceToHost,
                               h->stream));
    if (e)
        ILG_HIP(hipMemcpyAsync(e, h->mom + 2 * L, L * sizeof(int64_t), hipMemcpyDeviceToHost,
                               h->stream));
    rc = check_sticky(h);
    if (rc != ILG_OK)
        return rc;
    std::memset(out, 0, sizeof(*out));
    out->mass = res.mass;
    out->step = h->t;
    out->hash = res.hash;
    out->amplitude = res.sin_den > 0.0 ? res.sin_num / res.sin_den : 0.0;
    out->nk = nk;
    const double mf = (double)res.mass;
    for (uint32_t k = 0; k < nk; ++k)
        out->sk[k] = mf > 0.0 ? (res.sk_re[k] * res.sk_re[k] + res.sk_im[k] * res.sk_im[k]) / mf
                              : 0.0;
    return ILG_OK;
}

int ilg_state_hash(ilg_handle *h, uint64_t *out)
{
    if (!h || !out)
        return fail(ILG_E_INVALID, "null argument");
    ilg::DiagResult res;
    int rc = run_diag(h, false, 0, &res);
    if (rc != ILG_OK)
        return rc;
    rc = check_sticky(h);
    if (rc != ILG_OK)
        return rc;
    *out = res.hash;
    return ILG_OK;
}

int ilg_destroy(ilg_handle *h)
{
    if (!h)
        return ILG_OK;
    int rc = ILG_OK;
    if (hipStreamSynchronize(h->stream) == hipSuccess)
        rc = check_sticky(h);
    release(h);
    return rc;
}

}  // extern "C"

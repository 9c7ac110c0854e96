// Device-side Poisson sine initial state (the paper's initial condition,
// Results section: occupations drawn as Poisson variates with expectation
// w_i times the sine density profile N [1 + sin(2 pi x / L)], here with a
// general amplitude A: mean_i(x) = w_i (N + A sin(2 pi x / L))).
//
// Specification "init v1", chosen so that any IEEE-754 implementation draws
// the same counts: every floating-point step is one correctly rounded double
// operation (contraction into fused multiply-adds is switched off below, and
// no library transcendental is called).
//  * Nodes are x (1D) or x + Lx y (D2Q5), the profile runs along the column
//    x = node mod Lx; the node index is the counter word 0.
//  * sin(2 pi x / L): 8x = k L + rem in integers (octant k); t = rem / L for
//    even k, (L - rem) / L for odd k; a = t (pi/4); Taylor polynomials
//    S = a (1 + a^2 (s_1 + ... + a^2 s_8)), s_j = (-1)^j / (2j+1)!, and
//    C = 1 + a^2 (c_1 + ... + a^2 c_9), c_j = (-1)^j / (2j)!, in Horner form;
//    value S, C, C, S, -S, -C, -C, -S for k = 0..7.
//  * e^-m, 0 <= m <= 256: Cody-Waite reduction m = n ln 2 + r with
//    n = (int)(m log2 e + 1/2), r = (m - n ln2_hi) - n ln2_lo, then
//    e^-r = sum_{j<=17} (-r)^j / j! in Horner form, scaled by 2^-n.
//  * mean = w_i (N + A value); a mean <= 0 gives 0.  The mean is split into
//    P = max(1, ceil(mean / 256)) equal parts m = mean / P (a sum of
//    independent Poisson(m) is Poisson(mean)); part p draws word i of the
//    Philox4x32-10 block with key = init seed and counter
//    (x, p, realization, 2^31 + i / 4) (word i mod 4; the last counter word
//    keeps these blocks apart from the step's draws), U = (u + 1/2) 2^-32,
//    and returns the least k with
//    U <= F(k), where F(0) = f(0) = e^-m, f(k) = (f(k-1) m) / k and
//    F(k) = F(k-1) + f(k): the Poisson CDF by its recurrence (capped at 10^5).
// Coefficients 1/j! are 1 / j! with j! exact in double (j <= 18).
#include "ilg_internal.h"
#include "philox.h"

#pragma clang fp contract(off)

namespace ilg {

namespace {

constexpr double kPi4 = 0x1.921fb54442d18p-1;   // pi / 4
constexpr double kLog2e = 0x1.71547652b82fep+0;  // log2(e)
constexpr double kLn2Hi = 0x1.62e42feep-1;       // ln 2, upper bits
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33; // ln 2 - kLn2Hi
constexpr double kPartMean = 256.0;
constexpr uint32_t kMaxCount = 100000;

// 1 / j! as one correctly rounded division of an exact factorial.
constexpr double inv_fact(int j)
{
    double f = 1.0;
    for (int i = 2; i <= j; ++i)
        f = f * (double)i;
    return 1.0 / f;
}

__device__ double sin2pi_frac(uint32_t x, uint32_t L)
{
    const uint64_t ex = 8ull * x;
    const uint32_t k = (uint32_t)(ex / L);
    const uint64_t rem = ex % L;
    const double t = (double)((k & 1u) ? (uint64_t)L - rem : rem) / (double)L;
    const double a = t * kPi4;
    const double a2 = a * a;
    double hs = inv_fact(17);
    hs = -inv_fact(15) + a2 * hs;
    hs = inv_fact(13) + a2 * hs;
    hs = -inv_fact(11) + a2 * hs;
    hs = inv_fact(9) + a2 * hs;
    hs = -inv_fact(7) + a2 * hs;
    hs = inv_fact(5) + a2 * hs;
    hs = -inv_fact(3) + a2 * hs;
    hs = 1.0 + a2 * hs;
    const double S = a * hs;
    double hc = -inv_fact(18);
    hc = inv_fact(16) + a2 * hc;
    hc = -inv_fact(14) + a2 * hc;
    hc = inv_fact(12) + a2 * hc;
    hc = -inv_fact(10) + a2 * hc;
    hc = inv_fact(8) + a2 * hc;
    hc = -inv_fact(6) + a2 * hc;
    hc = inv_fact(4) + a2 * hc;
    hc = -inv_fact(2) + a2 * hc;
    const double C = 1.0 + a2 * hc;
    const bool cosine = ((k + 1u) & 2u) != 0;  // octants 1, 2, 5, 6
    const double v = cosine ? C : S;
    return k >= 4 ? -v : v;
}

__device__ double exp_neg(double m)
{
    const int n = (int)(m * kLog2e + 0.5);
    const double r = (m - (double)n * kLn2Hi) - (double)n * kLn2Lo;
    const double y = -r;
    double h = inv_fact(17);
    h = inv_fact(16) + y * h;
    h = inv_fact(15) + y * h;
    h = inv_fact(14) + y * h;
    h = inv_fact(13) + y * h;
    h = inv_fact(12) + y * h;
    h = inv_fact(11) + y * h;
    h = inv_fact(10) + y * h;
    h = inv_fact(9) + y * h;
    h = inv_fact(8) + y * h;
    h = inv_fact(7) + y * h;
    h = inv_fact(6) + y * h;
    h = inv_fact(5) + y * h;
    h = inv_fact(4) + y * h;
    h = inv_fact(3) + y * h;
    h = inv_fact(2) + y * h;
    h = 1.0 + y * h;
    h = 1.0 + y * h;
    return ldexp(h, -n);
}

__device__ uint32_t poisson_part(double m, uint32_t u)
{
    const double U = ((double)u + 0.5) * 0x1p-32;
    double f = exp_neg(m);
    double F = f;
    uint32_t k = 0;
    while (U > F && k < kMaxCount) {
        k += 1;
        f = (f * m) / (double)k;
        F = F + f;
    }
    return k;
}

// One thread per node; every velocity's count of that node.
template <typename T>
__global__ __launch_bounds__(256) void init_kernel(InitArgs a)
{
    T *out = reinterpret_cast<T *>(a.out);
    constexpr uint64_t kMax = (uint64_t)(T)~(T)0;
    bool overflow = false;
    for (uint64_t xx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; xx < a.length;
         xx += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t x = (uint32_t)xx;
        const double s = sin2pi_frac(x % a.width, a.width);
        const double rho = a.nave + a.amp * s;
        for (uint32_t i = 0; i < a.q; ++i) {
            const double mean = a.w[i] * rho;
            uint64_t n = 0;
            if (mean > 0.0) {
                const double pd = ceil(mean / kPartMean);
                const uint32_t parts = pd < 1.0 ? 1u : (uint32_t)pd;
                const double m = mean / (double)parts;
                for (uint32_t p = 0; p < parts; ++p) {
                    const uint4 b = philox4x32_10(x, p, a.realization, 0x80000000u + (i >> 2),
                                                  a.key0, a.key1);
                    const uint32_t w = i & 3u;
                    const uint32_t u = w == 0 ? b.x : (w == 1 ? b.y : (w == 2 ? b.z : b.w));
                    n += poisson_part(m, u);
                }
            }
            overflow |= n > kMax;
            out[(uint64_t)i * a.pitch + x] = (T)n;
        }
    }
    if (__builtin_amdgcn_ballot_w64(overflow) != 0ull && threadIdx.x % 64 == 0)
        atomicOr(a.err, 1u);
}

}  // namespace

hipError_t launch_init(int count_bytes, const InitArgs &a, hipStream_t stream)
{
    const uint32_t cus = (uint32_t)device_cu_count();
    uint32_t grid = (a.length + 255u) / 256u;
    if (grid > cus * 16u)
        grid = cus * 16u;
    if (grid == 0)
        return hipSuccess;
    if (count_bytes == 2)
        hipLaunchKernelGGL(init_kernel<uint16_t>, dim3(grid), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(init_kernel<uint32_t>, dim3(grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace ilg

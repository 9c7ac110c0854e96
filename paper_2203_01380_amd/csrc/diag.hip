// Diagnostics of a lattice state as wavefront reductions:
//   mass   = sum_{x,i} n_i(x)                                     (exact, u64)
//   hash   = sum_{x,i} splitmix64(((x q + i) << 32) ^ n_i(x)) mod 2^64  (exact)
//   A^LG   = sum_x sin(2 pi x/L) N(x) / sum_x sin^2(2 pi x/L)     (Results section)
//   S(k)   = |sum_x N(x) e^{-2 pi i k x/L}|^2 / sum_x N(x),  k = 1..nk      (FP64)
// and optionally the per-node raw moments rho = sum n_i, J = sum v_i n_i,
// E = sum v_i^2 n_i.  On a D2Q5 lattice x is the column (node mod Lx), the
// sums run over all nodes, J is the x momentum and E sums |v_i|^2.  Angles
// are reduced exactly in integers,
// (k x) mod L, before sincospi, so every term is accurate to a few ulp; the
// FP64 sums are deterministic (fixed grid, fixed tree).
#include "ilg_internal.h"

namespace ilg {

namespace {

constexpr int kDiagThreads = 256;
constexpr int kModesPerPass = 8;
constexpr int kSlots = 4 + 2 * 64;  // mass, hash, sin_num, sin_den, re[64], im[64]

__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename V>
__device__ __forceinline__ V block_sum(V v, V *scratch)
{
    for (int off = warpSize / 2; off > 0; off >>= 1)
        v += __shfl_down(v, off);
    const int lane = threadIdx.x % warpSize, wid = threadIdx.x / warpSize;
    __syncthreads();
    if (lane == 0)
        scratch[wid] = v;
    __syncthreads();
    V r = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x / warpSize); ++w)
            r += scratch[w];
    return r;  // valid in thread 0
}

template <typename T>
__device__ __forceinline__ uint64_t load_n(const T *s, uint64_t pitch, int i, uint32_t x)
{
    return s[(uint64_t)i * pitch + x];
}

template <typename T>
__global__ __launch_bounds__(kDiagThreads) void diag_kernel(DiagArgs a)
{
    __shared__ double sd[kDiagThreads / 64];
    __shared__ uint64_t su[kDiagThreads / 64];
    const T *s = reinterpret_cast<const T *>(a.state);
    const uint32_t L = a.length;        // nodes
    const uint32_t Lx = a.width;        // row length (angles along x)
    const int q = (int)a.q;
    uint64_t *part_u = reinterpret_cast<uint64_t *>(a.partials) + (size_t)blockIdx.x * kSlots;
    double *part_d = reinterpret_cast<double *>(part_u);

    uint64_t mass = 0, hash = 0;
    double sn = 0.0, sdn = 0.0;
    const uint32_t step = gridDim.x * blockDim.x;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < L; x += step) {
        uint64_t N = 0;
        int64_t J = 0, E = 0;
        for (int i = 0; i < q; ++i) {
            const uint64_t n = load_n(s, a.pitch, i, x);
            N += n;
            // x component and squared speed of velocity i
            const int v = (q == 2) ? (i == 0 ? -1 : 1)
                          : (q == 3) ? i - 1
                                     : (i == 0 ? -1 : (i == 4 ? 1 : 0));
            const int v2 = (q == 5) ? (i == 2 ? 0 : 1) : v * v;
            J += (int64_t)v * (int64_t)n;
            E += (int64_t)v2 * (int64_t)n;
            hash += splitmix64((((uint64_t)x * (uint64_t)q + (uint64_t)i) << 32) ^ n);
        }
        mass += N;
        if (a.rho) {
            a.rho[x] = (int64_t)N;
            a.j[x] = J;
            a.e[x] = E;
        }
        const uint32_t xc = Lx == L ? x : x % Lx;
        const double sv = sinpi(2.0 * (double)xc / (double)Lx);
        sn += sv * (double)N;
        sdn += sv * sv;
    }
    uint64_t r_mass = block_sum<uint64_t>(mass, su);
    uint64_t r_hash = block_sum<uint64_t>(hash, su);
    double r_sn = block_sum<double>(sn, sd);
    double r_sdn = block_sum<double>(sdn, sd);
    if (threadIdx.x == 0) {
        part_u[0] = r_mass;
        part_u[1] = r_hash;
        part_d[2] = r_sn;
        part_d[3] = r_sdn;
    }

    for (uint32_t k0 = 0; k0 < a.nk; k0 += kModesPerPass) {
        double re[kModesPerPass], im[kModesPerPass];
#pragma unroll
        for (int m = 0; m < kModesPerPass; ++m) {
            re[m] = 0.0;
            im[m] = 0.0;
        }
        for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < L; x += step) {
            uint64_t N = 0;
            for (int i = 0; i < q; ++i)
                N += load_n(s, a.pitch, i, x);
            const double Nd = (double)N;
#pragma unroll
            for (int m = 0; m < kModesPerPass; ++m) {
                const uint32_t k = k0 + m + 1;
                if (k <= a.nk) {
                    const uint64_t ang = ((uint64_t)k * (Lx == L ? x : x % Lx)) % Lx;
                    double sv, cv;
                    sincospi(2.0 * (double)ang / (double)Lx, &sv, &cv);
                    re[m] += Nd * cv;
                    im[m] -= Nd * sv;
                }
            }
        }
#pragma unroll
        for (int m = 0; m < kModesPerPass; ++m) {
            const double r1 = block_sum<double>(re[m], sd);
            const double r2 = block_sum<double>(im[m], sd);
            if (threadIdx.x == 0 && k0 + m < a.nk) {
                part_d[4 + k0 + m] = r1;
                part_d[4 + 64 + k0 + m] = r2;
            }
        }
    }
}

__global__ __launch_bounds__(kDiagThreads) void diag_finish_kernel(DiagArgs a, uint32_t nblocks)
{
    __shared__ double sd[kDiagThreads / 64];
    __shared__ uint64_t su[kDiagThreads / 64];
    const uint64_t *pu = reinterpret_cast<const uint64_t *>(a.partials);
    const double *pd = reinterpret_cast<const double *>(a.partials);
    DiagResult *res = reinterpret_cast<DiagResult *>(a.result);
    for (int slot = 0; slot < 4 + 2 * 64; ++slot) {
        const bool is_u = slot < 2;
        const bool used = slot < 4 || ((slot - 4) % 64) < (int)a.nk;
        if (!used)
            continue;
        uint64_t su_v = 0;
        double sd_v = 0.0;
        for (uint32_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
            if (is_u)
                su_v += pu[(size_t)b * kSlots + slot];
            else
                sd_v += pd[(size_t)b * kSlots + slot];
        }
        if (is_u) {
            const uint64_t r = block_sum<uint64_t>(su_v, su);
            if (threadIdx.x == 0) {
                if (slot == 0) res->mass = r;
                else res->hash = r;
            }
        } else {
            const double r = block_sum<double>(sd_v, sd);
            if (threadIdx.x == 0) {
                if (slot == 2) res->sin_num = r;
                else if (slot == 3) res->sin_den = r;
                else if (slot < 4 + 64) res->sk_re[slot - 4] = r;
                else res->sk_im[slot - 4 - 64] = r;
            }
        }
    }
}

}  // namespace

size_t diag_partials_bytes()
{
    return (size_t)kDiagBlocks * kSlots * sizeof(uint64_t);
}

hipError_t launch_diag(const DiagArgs &a, hipStream_t stream)
{
    uint32_t blocks = (a.length + kDiagThreads - 1) / kDiagThreads;
    if (blocks > (uint32_t)kDiagBlocks)
        blocks = kDiagBlocks;
    if (blocks == 0)
        blocks = 1;
    if (a.count_bytes == 2)
        hipLaunchKernelGGL(diag_kernel<uint16_t>, dim3(blocks), dim3(kDiagThreads), 0, stream, a);
    else
        hipLaunchKernelGGL(diag_kernel<uint32_t>, dim3(blocks), dim3(kDiagThreads), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kDiagThreads), 0, stream, a, blocks);
    return hipGetLastError();
}

}  // namespace ilg

// Exact fixed-point binomial CDF tables, built once per collision fraction on
// the host with multiword integers.
//
// For a removal probability p = P / 2^32 the scaled probabilities
//   s_m(i) = C(m, i) P^i (2^32 - P)^(m - i),  i = 0..m,   sum_i s_m(i) = 2^(32 m)
// satisfy s_m(i) = (2^32 - P) s_{m-1}(i) + P s_{m-1}(i-1).  The table entry is
//   T[m][j] = floor(2^32 * CDF_m(j)) = floor(sum_{i<=j} s_m(i) / 2^(32(m-1)))
// which, because the partial sum is below 2^(32 m), is limb m-1 of that sum.
#include <cstring>
#include <vector>

#include "ilg_internal.h"

namespace ilg {

namespace {

constexpr int kLimbs = kChunk + 1;  // s_m(i) < 2^(32 m) needs m limbs; one spare

struct Big {
    uint32_t limb[kLimbs];
};

}  // namespace

void build_binomial_table(uint64_t p, uint32_t *out)
{
    std::memset(out, 0, sizeof(uint32_t) * kTableEntries);
    if (p == 0 || p >= (uint64_t(1) << 32)) {
        // p = 1: every trial succeeds, CDF(j) = 0 for j < m (all zeros).
        // p = 0 has no representable table; callers special-case it.
        return;
    }
    const uint64_t P = p, Qc = (uint64_t(1) << 32) - p;
    std::vector<Big> cur(kChunk + 2), nxt(kChunk + 2);
    std::memset(cur.data(), 0, sizeof(Big) * cur.size());
    cur[0].limb[0] = 1;  // m = 0: s_0(0) = 1
    for (int m = 1; m <= kChunk; ++m) {
        // s_m(i) = Qc * s_{m-1}(i) + P * s_{m-1}(i-1), limb by limb
        for (int i = 0; i <= m; ++i) {
            uint64_t carry = 0;
            for (int k = 0; k < m; ++k) {
                uint64_t a = (i < m) ? cur[i].limb[k] : 0;
                uint64_t b = (i > 0) ? cur[i - 1].limb[k] : 0;
                // a*Qc + b*P + carry < 2^32 * (2^32 + ...) : split to stay in 64 bits
                uint64_t lo = a * Qc;            // < 2^64
                uint64_t acc = (lo & 0xFFFFFFFFu) + carry;
                uint64_t hi = lo >> 32;
                uint64_t lo2 = b * P;
                acc += lo2 & 0xFFFFFFFFu;
                hi += lo2 >> 32;
                nxt[i].limb[k] = static_cast<uint32_t>(acc);
                carry = hi + (acc >> 32);
            }
            nxt[i].limb[m] = static_cast<uint32_t>(carry);
            for (int k = m + 1; k < kLimbs; ++k)
                nxt[i].limb[k] = 0;
        }
        std::swap(cur, nxt);
        // partial sums; entry j is limb m-1 of sum_{i<=j} s_m(i)
        Big acc;
        std::memset(&acc, 0, sizeof(acc));
        uint32_t *row = out + (m - 1) * m / 2;
        for (int j = 0; j < m; ++j) {
            uint64_t c = 0;
            for (int k = 0; k <= m; ++k) {
                uint64_t s = uint64_t(acc.limb[k]) + cur[j].limb[k] + c;
                acc.limb[k] = static_cast<uint32_t>(s);
                c = s >> 32;
            }
            row[j] = acc.limb[m - 1];
        }
    }
}

void build_guide(const uint32_t *table, uint8_t *guide)
{
    for (int m = 1; m <= kChunk; ++m) {
        const uint32_t *row = table + (m - 1) * m / 2;
        for (int b = 0; b < kGuideBuckets; ++b) {
            const uint64_t edge = uint64_t(b) << (32 - kGuideBits);
            int c = 0;
            while (c < m && row[c] <= edge)
                ++c;
            guide[(m - 1) * kGuideBuckets + b] = static_cast<uint8_t>(c);
        }
    }
}

void pad_table(const uint32_t *packed, uint32_t *dev)
{
    for (uint32_t m = 1; m <= (uint32_t)kChunk; ++m) {
        const uint32_t *src = packed + (m - 1) * m / 2;
        uint32_t *dst = dev + dev_row_offset(m);
        for (uint32_t j = 0; j < m; ++j)
            dst[j] = src[j];
        for (int k = 0; k < kRowPad; ++k)
            dst[m + k] = 0xFFFFFFFFu;
    }
}

void build_table_set(uint64_t p, uint64_t p_rest, void *host_set)
{
    std::memset(host_set, 0, kTableSetBytes);
    uint32_t *tabs = reinterpret_cast<uint32_t *>(host_set);
    uint8_t *guides = reinterpret_cast<uint8_t *>(host_set) +
                      kTablesPerSet * kDevTableEntries * sizeof(uint32_t);
    const uint64_t ps[kTablesPerSet] = {p, uint64_t(1) << 31, p_rest};
    std::vector<uint32_t> packed(kTableEntries);
    for (int id = 0; id < kTablesPerSet; ++id) {
        if (ps[id] == 0)
            continue;
        build_binomial_table(ps[id], packed.data());
        build_guide(packed.data(), guides + id * kGuideEntries);
        pad_table(packed.data(), tabs + id * kDevTableEntries);
    }
}

}  // namespace ilg

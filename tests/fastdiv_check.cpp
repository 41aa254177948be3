// Host check of FastDiv (the multiply-high division the kernels use for site
// decoding): every quotient against the hardware division, for every divisor
// up to 4096, the divisors of the supported extents and products of them,
// and numerators covering [0, 2^16), multiples of d and their neighbours,
// and the top of the range below 2^31.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "../paper_1105_2279_amd/csrc/su3_device.hpp"

using qdpx::FastDiv;

static long long bad = 0, checked = 0;

static void check(uint32_t d, int n) {
    const FastDiv f = FastDiv::make(d);
    const int q = f.div(n);
    ++checked;
    if (q != (int)((uint32_t)n / d)) {
        if (bad < 10) std::printf("FAIL d=%u n=%d got %d want %u\n", d, n, q, (uint32_t)n / d);
        ++bad;
    }
}

int main() {
    std::vector<uint32_t> ds;
    for (uint32_t d = 1; d <= 4096; ++d) ds.push_back(d);
    const uint32_t extra[] = {4097, 6144, 8191, 8192, 12288, 65535, 65536, 110592, 131072, 221184, 1u << 20,
                              (1u << 20) + 1, 16777213, 1u << 27, (1u << 28) - 1, 1u << 28, 2147483647u};
    for (uint32_t d : extra) ds.push_back(d);
    uint64_t x = 88172645463325252ull;  // xorshift64 numerators
    for (uint32_t d : ds) {
        for (int n = 0; n < (d <= 64 ? 65536 : 4096); ++n) check(d, n);
        for (int k = 1; k < 64; ++k) {
            const uint64_t base = (uint64_t)d * (uint64_t)k * 977u;
            for (int e = -1; e <= 1; ++e) {
                const int64_t n = (int64_t)base + e;
                if (n >= 0 && n < 2147483648ll) check(d, (int)n);
            }
        }
        for (int k = 0; k < 256; ++k) {
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            check(d, (int)(x & 0x7fffffffu));
        }
        for (int n = 2147483647; n > 2147483647 - 64; --n) check(d, n);
    }
    std::printf("%lld checked, %lld wrong\n", checked, bad);
    return bad ? 1 : 0;
}

// Host check of the invariant-integer division the FP32-12 update kernel
// uses for a site's coordinates (div_magic in layout.h, applied as in
// geometry.h's div_by): every divisor up to 2^16 and a spread of larger ones,
// against the quotients x / d for the x at and around every multiple near
// the ends of the range, the ends themselves and pseudo-random x < 2^31.
// Prints the number of mismatches.
#include <cstdint>
#include <cstdio>
#include <initializer_list>

#include "layout.h"

static uint32_t div_by(uint32_t x, su3hb::DivMagic dm) { return uint32_t((uint64_t(x) * dm.m) >> dm.s); }

int main()
{
    uint64_t bad = 0, checked = 0, state = 88172645463325252ull;
    auto check = [&](uint32_t x, uint32_t d, su3hb::DivMagic dm) {
        if (x >= (1u << 31)) return;
        ++checked;
        if (div_by(x, dm) != x / d) {
            if (bad < 10) std::printf("mismatch x=%u d=%u\n", x, d);
            ++bad;
        }
    };
    auto run = [&](uint32_t d) {
        const su3hb::DivMagic dm = su3hb::div_magic(d);
        const uint32_t top = (1u << 31) - 1u;
        const uint32_t kmax = top / d;
        for (uint32_t k : {0u, 1u, 2u, kmax - 1u, kmax}) {
            const uint64_t base = uint64_t(k) * d;
            for (int o = -2; o <= 2; ++o) {
                const int64_t x = int64_t(base) + o;
                if (x >= 0) check(uint32_t(x), d, dm);
            }
            check(uint32_t(base + d - 1), d, dm);
        }
        check(top, d, dm);
        for (int j = 0; j < 64; ++j) {
            state ^= state << 13; state ^= state >> 7; state ^= state << 17;  // xorshift64
            check(uint32_t(state) & top, d, dm);
        }
    };
    for (uint32_t d = 1; d <= 65536u; ++d) run(d);
    for (uint64_t d = 65537; d < (1ull << 31); d = d * 3 / 2 + 7) run(uint32_t(d));
    std::printf("%llu mismatches in %llu checks\n", (unsigned long long)bad, (unsigned long long)checked);
    return bad ? 1 : 0;
}

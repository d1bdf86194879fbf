// Checks fast_div_multiplier against integer division: for many divisors,
// every quotient of x < bound at the largest bound the multiplier accepts
// (densely at the start and the end of the range), the refusal (m = 1) past
// that bound, and the d = 1 case.  The quotient is formed as the kernels
// form it: the high 32 bits of x m.
#include <cstdio>

#include "../../paper_2411_03501_amd/csrc/hjx_fastdiv.h"

static long quotient(long x, long d, unsigned m)
{
    if (m == 0) return x;
    if (m == 1) return x / d;
    return (long)(((unsigned long long)(unsigned)x * m) >> 32);
}

int main()
{
    long bad = 0, checked = 0;
    auto check_range = [&](long d, long bound) {
        const unsigned m = hjx::fast_div_multiplier(d, bound);
        if (d > 1 && m < 2) {
            ++bad;
            return;
        }
        for (long x = 0; x < bound && x < 200000; ++x, ++checked) bad += quotient(x, d, m) != x / d;
        for (long x = bound > 200000 ? bound - 200000 : 0; x < bound; ++x, ++checked) bad += quotient(x, d, m) != x / d;
        for (long x = 0; x < bound; x += 104729, ++checked) bad += quotient(x, d, m) != x / d;
    };
    for (long d = 1; d <= 3000; ++d) {
        long bound = (long)(0x100000000ull / (unsigned long long)d);
        if (bound > 0x7fffffffL) bound = 0x7fffffffL;
        check_range(d, bound);
    }
    for (long d = 3001; d < 100000000L; d = d * 5 / 4 + 13) check_range(d, (long)(0x100000000ull / (unsigned long long)d));
    // past the bound the multiplier is refused and the quotient is a division
    for (long d = 2; d < 100000; d = d * 3 + 1) {
        const long bound = (long)(0x100000000ull / (unsigned long long)d) + 1;
        ++checked;
        bad += hjx::fast_div_multiplier(d, bound) != 1;
    }
    bad += hjx::fast_div_multiplier(1, 0x7fffffffL) != 0;
    std::printf("fastdiv: %ld checked, %ld wrong\n", checked, bad);
    return bad != 0;
}

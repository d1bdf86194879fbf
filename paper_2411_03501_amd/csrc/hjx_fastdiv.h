// Division by a divisor fixed for a whole launch, as a multiply-high: the
// host picks the multiplier, the kernels apply it (udiv in hjx_internal.h).
// Plain C++, so that the host side can be checked on its own.
#pragma once

namespace hjx {

// Multiplier for x / d with 0 <= x < bound:
//   0 when d <= 1 (the quotient is x itself);
//   1 when bound * d > 2^32 (no exact multiplier of this form: divide);
//   otherwise m = ceil(2^32 / d), and x / d = (x * m) >> 32 exactly.
// Why exact: m d = 2^32 + e with 0 <= e < d, so x m / 2^32 =
// x / d + x e / (d 2^32), and the second term is below 1 / d because
// x e < x d < bound d <= 2^32; it cannot carry the fraction of x / d, at most
// 1 - 1/d, past the next integer.
inline unsigned fast_div_multiplier(long d, long bound)
{
    if (d <= 1) return 0;
    if ((unsigned long long)bound * (unsigned long long)d > 0x100000000ull) return 1;
    return (unsigned)((0x100000000ull + (unsigned long long)d - 1) / (unsigned long long)d);
}

}  // namespace hjx

// Natural logarithm of the temperature for the Arrhenius rates, written out from the series
//
//   log(1 + f) = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),   s = f / (2 + f),
//
// after splitting x = 2^e m with m in [sqrt(1/2), sqrt(2)), f = m - 1 (exact), so that
// |s| <= 0.1716 and ten terms leave a relative truncation below 1e-18.  The sum is taken
// as f - s (f - R) with R = 2 s^2 (1/3 + s^2/5 + ... + s^18/21), so that the rounding of s
// only reaches the small correction term; e ln 2 is added with ln 2 split in a 32-bit head
// (e times it is exact) and the rest.  About 1 ulp over the positive doubles (a CPU test
// compares it with the C library's log), against about 110 instructions for the general
// library routine, which also serves arguments this kernel never passes.  0 gives -inf,
// negative arguments and NaN give NaN, +inf gives +inf.  Host and device code alike.
#pragma once

#include <stdint.h>
#include <string.h>

#ifdef __HIPCC__
#define ZB_LOG_FN __host__ __device__ __forceinline__
#else
#define ZB_LOG_FN inline
#endif

namespace zbm {

ZB_LOG_FN double log_series(double x)
{
    // x = 2^e m; subnormal arguments are scaled into the normal range first
    const bool sub = x < 0x1p-1022;
    const double xs = sub ? x * 0x1p54 : x;
    uint64_t b;
    memcpy(&b, &xs, sizeof b);
    int e = (int)((b >> 52) & 0x7ff) - 1023 - (sub ? 54 : 0);
    b = (b & 0x000fffffffffffffull) | 0x3ff0000000000000ull;   // m in [1, 2)
    double m;
    memcpy(&m, &b, sizeof m);
    const bool high = m > 0x1.6a09e667f3bcdp+0;                // sqrt(2)
    m = high ? 0.5 * m : m;
    e += high ? 1 : 0;
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double p = 0x1.8618618618618p-5;                 // 1/21
    p = __builtin_fma(p, z, 0x1.af286bca1af28p-5);   // 1/19
    p = __builtin_fma(p, z, 0x1.e1e1e1e1e1e1ep-5);   // 1/17
    p = __builtin_fma(p, z, 0x1.1111111111111p-4);   // 1/15
    p = __builtin_fma(p, z, 0x1.3b13b13b13b14p-4);   // 1/13
    p = __builtin_fma(p, z, 0x1.745d1745d1746p-4);   // 1/11
    p = __builtin_fma(p, z, 0x1.c71c71c71c71cp-4);   // 1/9
    p = __builtin_fma(p, z, 0x1.2492492492492p-3);   // 1/7
    p = __builtin_fma(p, z, 0x1.999999999999ap-3);   // 1/5
    p = __builtin_fma(p, z, 0x1.5555555555555p-2);   // 1/3
    const double R = 2.0 * z * p;
    const double lm = __builtin_fma(-s, f - R, f);  // log(m)
    const double ed = (double)e;
    const double r = __builtin_fma(ed, 0x1.62e42fee00000p-1,     // ln 2, first 32 bits
                                   __builtin_fma(ed, 0x1.a39ef35793c76p-33, lm));   // the rest
    if (x > 0.0 && x < __builtin_inf()) return r;
    if (x == 0.0) return -__builtin_inf();
    return x > 0.0 ? x : __builtin_nan("");
}

}  // namespace zbm

// Double-precision reciprocal, square root and k-th root from approximate starting values,
// for the step control of the burn kernels (WRMS norms and step-size factors), and the
// reciprocal also for the pivots, 1/T of the rates and the error weights.  The device
// code starts from the hardware approximations (v_rcp_f64, v_sqrt_f64: about 2^-23
// relative; the FP32 log2 and exp2 for the root) and refines them with Newton steps to
// about 1 ulp, so that step sizes and accept/reject decisions agree with the exact formulas
// as closely as the library routines would, at a fraction of their instructions.  The
// starting values are arguments, so a CPU test can feed perturbed ones.  Host and device.
#pragma once

#ifdef __HIPCC__
#define ZB_SM_FN __host__ __device__ __forceinline__
#else
#define ZB_SM_FN inline
#endif

namespace zbm {

// 1/d from r0 within 2^-20 relative: two Newton steps (error ~ e^2, then ~ e^4).
ZB_SM_FN double recip_from(double d, double r0)
{
    double e = __builtin_fma(-d, r0, 1.0);
    const double r = __builtin_fma(r0, e, r0);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// sqrt(x) for finite x > 0 from y0 ~ sqrt(x) and r0 ~ 1/y0, both within 2^-20 relative:
// two steps y += (x - y^2) / (2 y) with the approximate 1/(2 y0).
ZB_SM_FN double sqrt_from(double x, double y0, double r0)
{
    const double h = 0.5 * r0;
    const double y = __builtin_fma(__builtin_fma(-y0, y0, x), h, y0);
    return __builtin_fma(__builtin_fma(-y, y, x), h, y);
}

// x^(1/k) for finite x > 0 and 1 <= k <= 6, from y0 within 2^-16 relative: two Newton steps
// on y^k = x, y += (x - y^k) / (k y^(k-1)).  The first takes the divisor's reciprocal from
// rcp (an approximation within 2^-20 relative; the error then falls as e^2 + e 2^-20, to
// about 1e-9), the second refines it (the error falls as e^2, to rounding).
template <class Rcp>
ZB_SM_FN double root_from(double x, int k, double y0, Rcp rcp)
{
    double y = y0;
    for (int it = 0; it < 2; ++it) {
        double p = 1.0;   // y^(k-1)
        for (int j = 1; j < 6; ++j) p = j < k ? p * y : p;
        const double num = __builtin_fma(-p, y, x);
        const double d = (double)k * p;
        const double r = it == 0 ? rcp(d) : recip_from(d, rcp(d));
        y = __builtin_fma(num, r, y);
    }
    return y;
}

}  // namespace zbm

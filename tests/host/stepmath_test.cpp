// CPU test of the step-control refinements (zb_stepmath.h): from starting values off by up
// to the error bounds the kernels assume for the hardware approximations (2^-20 for the
// reciprocal and square root, 2^-16 for the FP32 root), the results must be within about
// 1 ulp of the exact values (x87 extended precision as the reference).
#include <math.h>
#include <stdio.h>

#include <random>

#include "zb_stepmath.h"

static double ulps(double got, long double ref)
{
    const double r = (double)ref;
    const double u = nextafter(fabs(r), INFINITY) - fabs(r);
    return (double)(fabsl((long double)got - ref) / u);
}

int main()
{
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    auto pert = [&](double v, double rel) { return v * (1.0 + rel * u(g)); };
    // the kernels' reciprocal inside the root: an approximation within 2^-20
    auto rcp = [&](double d) { return pert(1.0 / d, 0x1p-20); };
    double wr = 0, ws = 0, wk = 0;
    for (int i = 0; i < 2000000; ++i) {
        const double x = exp2(-1000.0 + 2000.0 * (0.5 + 0.5 * u(g)));
        wr = fmax(wr, ulps(zbm::recip_from(x, pert(1.0 / x, 0x1p-20)), 1.0L / (long double)x));
        const double y0 = pert(sqrt(x), 0x1p-20);
        ws = fmax(ws, ulps(zbm::sqrt_from(x, y0, pert(1.0 / y0, 0x1p-20)), sqrtl((long double)x)));
    }
    // the roots of the step-size factors: b E over the FP32 normal range, k = 1..6
    for (int i = 0; i < 3000000; ++i) {
        const double x = exp2(-126.0 + 253.0 * (0.5 + 0.5 * u(g)));
        const int k = 1 + i % 6;
        const long double ref = powl((long double)x, 1.0L / k);
        const double y0 = pert((double)ref, 0x1p-16);
        wk = fmax(wk, ulps(zbm::root_from(x, k, y0, rcp), ref));
    }
    // the whole root as the kernels take it: x = 2^(k j) xs, an FP32 start for xs, the
    // refinement, 2^j back; every positive double, subnormals included
    auto kth_root = [&](double x, int k) {
        int e;
        frexp(x, &e);
        const float rk = (float)pert(1.0 / k, 0x1p-22);
        const int j = (int)((float)e * rk);
        const double xs = ldexp(x, -k * j);
        const double y0 = (double)exp2f(log2f((float)xs) * rk);
        return ldexp(zbm::root_from(xs, k, y0, rcp), j);
    };
    double wa = 0;
    for (int i = 0; i < 3000000; ++i) {
        const double x = exp2(-1074.0 + 2097.0 * (0.5 + 0.5 * u(g)));
        const int k = 1 + i % 6;
        wa = fmax(wa, ulps(kth_root(x, k), powl((long double)x, 1.0L / k)));
    }
    printf("recip %.3f ulp, sqrt %.3f ulp, k-th root %.3f ulp, scaled k-th root %.3f ulp\n", wr, ws, wk, wa);
    if (!(wr <= 1.0 && ws <= 1.0 && wk <= 1.5 && wa <= 1.5)) {
        printf("stepmath check failed\n");
        return 1;
    }
    printf("stepmath ok\n");
    return 0;
}

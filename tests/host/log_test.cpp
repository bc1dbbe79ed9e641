// CPU test of the series logarithm the burn kernels use for the Arrhenius rates
// (zb_log.h): error in units in the last place against the x87 extended-precision logl,
// over the whole range of positive doubles, the temperatures of the workloads, arguments
// next to 1 and the subnormals, plus the special values.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>

#include "zb_log.h"

static double ulp_err(double x)
{
    const double got = zbm::log_series(x);
    const long double ref = logl((long double)x);
    const double u = nextafter(fabs((double)ref), INFINITY) - fabs((double)ref);
    return (double)fabsl((long double)got - ref) / u;
}

int main()
{
    std::mt19937_64 g(12345);
    double worst = 0.0, worst_x = 0.0, all = 0.0;
    auto run = [&](double x) {
        const double e = ulp_err(x);
        if (e > worst) {
            worst = e;
            worst_x = x;
        }
    };
    std::uniform_real_distribution<double> u(0.0, 1.0);
    auto range = [&](const char *name, int n, auto gen) {
        worst = 0.0;
        for (int i = 0; i < n; ++i) run(gen(i));
        printf("%-28s worst %.3f ulp at %a\n", name, worst, worst_x);
        all = fmax(all, worst);
    };
    range("all positive doubles", 2000000, [&](int) { return exp2(-1074.0 + 2098.0 * u(g)); });
    range("temperatures 30..1e5", 2000000, [&](int) { return exp(log(30.0) + (log(1e5) - log(30.0)) * u(g)); });
    range("next to 1", 1000000, [&](int) { return 1.0 + (u(g) - 0.5) * 1e-3; });
    range("next to the sqrt(2) split", 1000000,
          [&](int) { return 0x1.6a09e667f3bcdp+0 * (1.0 + (u(g) - 0.5) * 1e-6); });
    range("subnormals", 200000, [&](int i) { return ldexp((double)(i + 1), -1074); });
    worst = 0.0;
    const double a = 0.6931471805599453;
    run(1.0); run(2.0); run(0.5); run(a); run(1e300); run(1.7976931348623157e308); run(2.2250738585072014e-308);
    all = fmax(all, worst);
    int bad = 0;
    if (!(all <= 1.2)) bad = 1;
    if (zbm::log_series(1.0) != 0.0) bad = 2;
    if (!(zbm::log_series(0.0) == -INFINITY)) bad = 3;
    if (!(zbm::log_series(-0.0) == -INFINITY)) bad = 4;
    if (!isnan(zbm::log_series(-1.0))) bad = 5;
    if (!isnan(zbm::log_series(NAN))) bad = 6;
    if (!(zbm::log_series(INFINITY) == INFINITY)) bad = 7;
    if (!isnan(zbm::log_series(-INFINITY))) bad = 8;
    if (bad) {
        printf("log check %d failed\n", bad);
        return 1;
    }
    printf("log ok\n");
    return 0;
}

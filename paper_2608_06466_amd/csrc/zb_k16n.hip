// Instantiations of the burn kernel: 16, 8, double, 0, 16, 8, float, 1, 16, 4, double, 0, 16, 4, float, 1 (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_16n(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_K(16, 8, double, 0),
        ZB_K(16, 8, float, 1),
        ZB_K(16, 4, double, 0),
        ZB_K(16, 4, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

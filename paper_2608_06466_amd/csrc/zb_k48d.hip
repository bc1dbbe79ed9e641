// Instantiations of the burn kernel: 48, 64, double, 0 (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_48d(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_K(48, 64, double, 0),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

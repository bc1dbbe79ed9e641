// Instantiations of the burn kernel: 48, 64, float, 1 (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_48f(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_K(48, 64, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

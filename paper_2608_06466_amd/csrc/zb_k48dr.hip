// Instantiations of the burn kernel with the VODE-style Jacobian/LU reuse (jac_policy 1):
// 48, 64, double, 0 (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_48dr(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KR(48, 64, double, 0),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

// Instantiations of the burn kernel with the VODE-style Jacobian/LU reuse (jac_policy 1):
// 24, 32, double, 0, 24, 32, float, 1 (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_24r(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KR(24, 32, double, 0),
        ZB_KR(24, 32, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

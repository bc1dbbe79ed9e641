// Instantiations of the burn kernel with the VODE-style Jacobian/LU reuse (jac_policy 1):
// 4, 1, double, 0, 4, 4, double, 0, 4, 1, float, 1, 4, 4, float, 1, 8, 8, double, 0, 8, 8, float, 1 (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_04r(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KR(4, 1, double, 0),
        ZB_KR(4, 4, double, 0),
        ZB_KR(4, 1, float, 1),
        ZB_KR(4, 4, float, 1),
        ZB_KR(8, 8, double, 0),
        ZB_KR(8, 8, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

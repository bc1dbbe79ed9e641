// Instantiations of the burn kernel for 22-variable networks with the Jacobian/LU reuse, rows not padded:
// (22, 32, double); (22, 32, float) (rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_22r(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KR(22, 32, double, 0),
        ZB_KR(22, 32, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

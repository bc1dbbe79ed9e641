// Instantiations of the burn kernel for the variable-coefficient BDF form with the VODE-style Jacobian/LU reuse:
// (24, 32, double); (24, 32, float); (32, 32, double); (32, 32, float) (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_vr_c(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KVR(24, 32, double, 0),
        ZB_KVR(24, 32, float, 1),
        ZB_KVR(32, 32, double, 0),
        ZB_KVR(32, 32, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

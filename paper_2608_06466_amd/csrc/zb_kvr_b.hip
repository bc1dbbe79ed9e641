// Instantiations of the burn kernel for the variable-coefficient BDF form with the VODE-style Jacobian/LU reuse:
// (16, 16, double); (16, 16, float) (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_vr_b(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KVR(16, 16, double, 0),
        ZB_KVR(16, 16, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

// Instantiations of the burn kernel for the variable-coefficient BDF form with the VODE-style Jacobian/LU reuse:
// (48, 64, double) (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_vr_d(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KVR(48, 64, double, 0),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

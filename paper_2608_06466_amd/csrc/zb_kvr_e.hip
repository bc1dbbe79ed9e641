// Instantiations of the burn kernel for the variable-coefficient BDF form with the VODE-style Jacobian/LU reuse:
// (48, 64, float) (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_vr_e(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KVR(48, 64, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

// Instantiations of the burn kernel for the variable-coefficient BDF form with a Jacobian every step:
// (48, 64, double) (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_v_d(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KV(48, 64, double, 0),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

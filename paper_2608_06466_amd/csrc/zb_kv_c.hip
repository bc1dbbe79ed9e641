// Instantiations of the burn kernel for the variable-coefficient BDF form with a Jacobian every step:
// (24, 32, double); (24, 32, float); (32, 32, double); (32, 32, float) (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_v_c(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KV(24, 32, double, 0),
        ZB_KV(24, 32, float, 1),
        ZB_KV(32, 32, double, 0),
        ZB_KV(32, 32, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

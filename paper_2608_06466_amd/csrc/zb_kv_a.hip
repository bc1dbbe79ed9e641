// Instantiations of the burn kernel for the variable-coefficient BDF form with a Jacobian every step:
// (4, 1, double); (4, 4, double); (4, 1, float); (4, 4, float); (8, 8, double); (8, 8, float) (padded rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_v_a(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KV(4, 1, double, 0),
        ZB_KV(4, 4, double, 0),
        ZB_KV(4, 1, float, 1),
        ZB_KV(4, 4, float, 1),
        ZB_KV(8, 8, double, 0),
        ZB_KV(8, 8, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

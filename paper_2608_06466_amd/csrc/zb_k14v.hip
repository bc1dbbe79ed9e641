// Instantiations of the burn kernel for 14-variable networks, variable-coefficient form, rows not padded:
// (14, 16, double); (14, 16, float) (rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_14v(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KV(14, 16, double, 0),
        ZB_KV(14, 16, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

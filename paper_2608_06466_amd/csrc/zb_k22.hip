// Instantiations of the burn kernel for 22-variable networks (21 species and T), rows not padded:
// (22, 32, double); (22, 32, float) (rows, lanes per zone, LU type).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_22(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_K(22, 32, double, 0),
        ZB_K(22, 32, float, 1),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

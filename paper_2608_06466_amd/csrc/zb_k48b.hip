// Instantiations of the burn kernel with the blocked matrix-core FP32 LU, for networks of
// 33 to 48 variables on a whole wave: fixed- and variable-coefficient BDF, Jacobian every step.
#include "zb_burn_kernel.h"

namespace zb {

int kernels_48b(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KB(48, 64),
        ZB_KVB(48, 64),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

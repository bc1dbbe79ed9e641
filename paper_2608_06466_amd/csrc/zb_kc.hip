// Instantiations of the burn kernel with the Runge-Kutta-Chebyshev integrator (FP64; the
// method has no iteration matrix): (4,1), (4,4), (8,8), (16,16), (24,32), (32,32), (48,64).
#include "zb_burn_kernel.h"

namespace zb {

int kernels_rkc(const KernelInfo **out)
{
    static const KernelInfo t[] = {
        ZB_KC(4, 1), ZB_KC(4, 4), ZB_KC(8, 8), ZB_KC(16, 16), ZB_KC(24, 32), ZB_KC(32, 32),
        ZB_KC(48, 64),
    };
    *out = t;
    return (int)(sizeof(t) / sizeof(t[0]));
}

}  // namespace zb

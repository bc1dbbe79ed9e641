// Small support kernels of libzoneburn and the table of burn-kernel instantiations
// (each zb_k*.hip file instantiates some of them, so they compile in parallel).

#include <vector>

#include "zb_internal.h"

namespace zb {

int kernels_04(const KernelInfo **out);
int kernels_16(const KernelInfo **out);
int kernels_14(const KernelInfo **out);
int kernels_48b(const KernelInfo **out);
int kernels_14r(const KernelInfo **out);
int kernels_14v(const KernelInfo **out);
int kernels_14vr(const KernelInfo **out);
int kernels_22(const KernelInfo **out);
int kernels_22r(const KernelInfo **out);
int kernels_16n(const KernelInfo **out);
int kernels_24(const KernelInfo **out);
int kernels_32(const KernelInfo **out);
int kernels_48d(const KernelInfo **out);
int kernels_48f(const KernelInfo **out);
int kernels_04r(const KernelInfo **out);
int kernels_v_a(const KernelInfo **out);
int kernels_v_b(const KernelInfo **out);
int kernels_v_c(const KernelInfo **out);
int kernels_v_d(const KernelInfo **out);
int kernels_v_e(const KernelInfo **out);
int kernels_vr_a(const KernelInfo **out);
int kernels_vr_b(const KernelInfo **out);
int kernels_vr_c(const KernelInfo **out);
int kernels_vr_d(const KernelInfo **out);
int kernels_vr_e(const KernelInfo **out);
int kernels_16r(const KernelInfo **out);
int kernels_24r(const KernelInfo **out);
int kernels_32r(const KernelInfo **out);
int kernels_48dr(const KernelInfo **out);
int kernels_48fr(const KernelInfo **out);
int kernels_rkc(const KernelInfo **out);

__global__ void reset_kernel(unsigned long long *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_reset(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(reset_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

int kernel_table(const KernelInfo **out)
{
    static const std::vector<KernelInfo> table = [] {
        std::vector<KernelInfo> t;
        auto add = [&](int (*f)(const KernelInfo **)) {
            const KernelInfo *p = nullptr;
            int n = f(&p);
            t.insert(t.end(), p, p + n);
        };
        add(kernels_04);
        add(kernels_16);
        add(kernels_14);
        add(kernels_48b);
        add(kernels_14r);
        add(kernels_14v);
        add(kernels_14vr);
        add(kernels_22);
        add(kernels_22r);
        add(kernels_16n);
        add(kernels_24);
        add(kernels_32);
        add(kernels_48d);
        add(kernels_48f);
        add(kernels_04r);
        add(kernels_16r);
        add(kernels_24r);
        add(kernels_32r);
        add(kernels_48dr);
        add(kernels_48fr);
        add(kernels_v_a);
        add(kernels_v_b);
        add(kernels_v_c);
        add(kernels_v_d);
        add(kernels_v_e);
        add(kernels_vr_a);
        add(kernels_vr_b);
        add(kernels_vr_c);
        add(kernels_vr_d);
        add(kernels_vr_e);
        add(kernels_rkc);
        return t;
    }();
    *out = table.data();
    return (int)table.size();
}

}  // namespace zb

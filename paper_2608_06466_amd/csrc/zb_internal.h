// Internal types shared by the device code and the host runtime of libzoneburn.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zb {

constexpr int QMAX = 5;      // highest BDF order
constexpr int NVMAX = 64;    // largest number of integrated variables
constexpr int RMAX = 4096;   // largest number of reactions

// A network as the kernels read it.  Built once per network by the host.
//  rct[r] = (a, b, c, d): reactants a, b and products c, d (-1 when absent).
//  par[r] = (lnA, n, E, q).
//  inv[i][e], for every reaction r whose net stoichiometry nu_ir in species i is
//              non-zero: .x = r | nu_ir << 16 (nu_ir a signed 16-bit field, read with
//              an arithmetic shift), .y = a_r | (b_r + 1) << 8 (the reactant columns
//              the row's Jacobian entries go to, so no second lookup is needed);
//              entries with nu = 0 (.x = 0) pad the row.
//  The row length inv_len is even (the kernels read two entries at a time).
struct DevNet {
    int ns, nv, thermal, nr;
    int inv_len;
    const int4 *rct;
    const double4 *par;
    const int2 *inv;
};

// One run of zones that share a network and tolerances.
struct Segment {
    DevNet net;
    double *state;          // [zones][ns+1]
    const double *scale;    // [zones][nr] or null
    const double *source;   // [zones][ns+1] constant term added to f, or null
    int32_t *status;        // [zones] or null
    int32_t *stats;         // [zones][7] or null
    int64_t zones;
    double dt, rtol, atol;
};

constexpr int MAXSEG = 8;

struct BurnArgs {
    Segment seg[MAXSEG];
    int nseg;
    int max_nr;                    // largest reaction count of the segments (sizes the LDS)
    int max_steps;
    int retry, retry_max_steps;    // zone-by-zone retry of failed zones (0: off)
    int retry_jac;                 // retry Jacobian: 0 analytic, 1 finite differences
    double retry_rtol, retry_atol;
    unsigned long long *queue;     // [nseg] next zone of each segment (zeroed before the launch)
    unsigned long long *nfail;     // zones that ended with a non-OK status
    int rates_lds;                 // 1: per-reaction rate factors kept in LDS (some segment
                                   // has rate scales or a network without temperature)
    unsigned long long *fb;        // FP64 fallback: MAXSEG counters, then MAXSEG x FB_CAP zones
    int fb_mode;                   // 0 off; 1 the mixed run lists its failed zones;
                                   // 2 the FP64 run burns the listed zones
};

// FP64 fallback lists: zones per segment and launch (further failed zones keep their
// mixed-precision status), and the device words of one launch's lists.
constexpr int FB_CAP = 1024;
constexpr int FB_STRIDE = MAXSEG * (1 + FB_CAP);

// Kernel methods (a template parameter of the burn kernel, KernelInfo.jac on the host):
// fixed-coefficient BDF with the Jacobian every step or reused, RKC, the same two for the
// variable-coefficient BDF, and the two every-step BDF forms with the blocked matrix-core LU.
enum { METHOD_BDF = 0, METHOD_BDF_REUSE = 1, METHOD_RKC = 2, METHOD_BDF_VC = 3,
       METHOD_BDF_VC_REUSE = 4, METHOD_BDF_BLU = 5, METHOD_BDF_VC_BLU = 6 };
__host__ __device__ constexpr bool method_vc(int m)
{
    return m == METHOD_BDF_VC || m == METHOD_BDF_VC_REUSE || m == METHOD_BDF_VC_BLU;
}
__host__ __device__ constexpr int method_jac(int m)
{
    return (m == METHOD_BDF_REUSE || m == METHOD_BDF_VC_REUSE) ? 1 : 0;
}
__host__ __device__ constexpr bool method_blocked_lu(int m)
{
    return m == METHOD_BDF_BLU || m == METHOD_BDF_VC_BLU;
}

// The history copy of a step attempt (the Nordsieck array before the prediction, restored
// after a failed attempt) is held in registers in the mixed 14-row kernels that run three
// waves a SIMD (a Jacobian every step, and the two reuse forms) and the mixed 22-row one
// with a Jacobian every step (three waves as well: 14 % faster), whose LDS bounds the
// workgroups a CU holds (12 without the copy's 84 doubles a zone, 11 with them: 5 % faster
// on the 2^20-zone headline, bitwise the same).  Elsewhere registers bound them, and the
// copy stays in LDS (in registers it made the batched FP64 burn 7 % slower, the 48-row
// kernel spilling more).
__host__ __device__ constexpr bool hist_regs(int nvp, int L, bool mixed, int method)
{
    return (nvp == 14 && L == 16 && mixed &&
            (method == METHOD_BDF || method == METHOD_BDF_REUSE || method == METHOD_BDF_VC_REUSE)) ||
           (nvp == 22 && L == 32 && mixed && method == METHOD_BDF);
}

// Per-group LDS layout (in doubles).  Everything a zone group exchanges lives here.
struct LdsLayout {
    int cnt, zs, ybuf, wbuf, prow, ks, rx, jbuf, vc, total;
};

// Variable-coefficient BDF slots (kernels of that form only): the accepted step sizes,
// newest first, their count, the corrector coefficients l_0..l_QMAX of the current attempt
// and its error divisor.
constexpr int VC_HIST = 0, VC_COUNT = QMAX, VC_L = QMAX + 1, VC_EDIV = 2 * QMAX + 2,
              VC_SLOTS = 2 * QMAX + 4;

// The Jacobian rows are kept in FP32 in the mixed 48-row kernels: they only feed the
// iteration matrix, which those kernels round to FP32 anyway, and the halved buffer lets
// eight zones share a CU (five with FP64 rows) at 150 reactions.
__host__ __device__ constexpr bool jac_f32(int nvp, bool mixed) { return mixed && nvp >= 48; }

// The trimmed layout of the kernels with one row a lane in groups of 16 lanes or more (and
// FP64 Jacobian rows): the history copy has one slot per row instead of per lane, there is
// no pivot-row buffer (pivot rows are read from registers), and the per-reaction rate
// factors take no space when they are all 1.  It is for the classes whose LDS, not their
// registers, bounds the zones a CU holds: the FP64 48-row kernel (five of a possible eight
// at 150 reactions, six trimmed), and the mixed 14-row one at three waves a SIMD (10
// workgroups a CU, 11 trimmed: 7 % faster on the 2^20-zone headline, bitwise the same).
__host__ __device__ constexpr bool lds_trim(int L, int rpl, bool jf32)
{
    return L >= 16 && rpl == 1 && !jf32;
}

// L lanes per zone with rpl rows each.  rates: the per-reaction rate factors (the zone's rate
// scales, or a network's constant rates when it has no temperature) are needed; without
// rate scales and with a temperature variable they are all 1.
__host__ __device__ inline LdsLayout lds_layout(int nvp, int L, int rpl, int nr, bool vc,
                                                bool jf32, bool rates, bool hregs)
{
    const bool trim = lds_trim(L, rpl, jf32);
    LdsLayout o;
    int p = 0;
    o.cnt = p;  p += 4;               // counters of a zone's first run while it is retried
    o.zs = p;   p += hregs ? 0 : (QMAX + 1) * (trim ? nvp : L * rpl);
    o.ybuf = p; p += nvp;
    o.wbuf = p; p += nvp;
    o.prow = p; p += trim ? 0 : nvp;
    o.ks = p;   p += (trim && !rates) ? 0 : nr;
    p = (p + 1) & ~1;
    o.rx = p;   p += 4 * nr;          // w, dw/dYa, dw/dYb, dw/dT: four columns of nr
    o.jbuf = p;                       // Jacobian rows with an odd stride (no bank conflicts)
    p += jf32 ? (nvp * (nvp + 1) + 1) / 2 : nvp * (nvp + 1);
    o.vc = p;   p += vc ? VC_SLOTS : 0;
    // One or two lanes a zone: consecutive zones' areas start an odd number of doubles apart,
    // so a wave's same-slot accesses spread over all LDS banks (a stride of a multiple of 8
    // dwords put the 64 zones of a wave on 8 banks).  Wider groups keep an even stride (odd
    // raised the 4-lane kernels' bank conflicts from 0.02 to 0.6 per LDS-active cycle).
    o.total = L < 4 ? (p | 1) : ((p + 1) & ~1);
    return o;
}

// Kernel entry points, one per (padded size, lanes per zone, LU precision).
struct KernelInfo {
    int nvp;          // padded number of variables the kernel handles (nv <= nvp)
    int lanes;        // lanes per zone
    int mixed;        // 0: FP64 LU, 1: FP32 LU
    int jac;          // method (METHOD_*)
    const void *fn;   // __global__ function
};

int kernel_table(const KernelInfo **out);
hipError_t launch_reset(unsigned long long *p, int n, hipStream_t s);

}  // namespace zb

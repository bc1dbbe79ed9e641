// Per-zone BDF burn kernels for gfx950 (device code; instantiated by zb_k*.hip).
//
// Mapping.  A zone is integrated by a group of L lanes of one wavefront
// (L = 1, 2, ..., 64; 64/L zones per wave).  Row i of the iteration matrix
// M = I - gamma J, and component i of every per-zone vector, belong to lane
// i % L of the group (local slot i / L), so M lives in registers with static
// column indices.  The zone's scalars (t, h, q, counters) are replicated in
// the group's lanes and stay bitwise identical because every value they come
// from is a group-wide reduction with the same result in each lane.
//
// Exchange.  Group reductions use DPP (quad_perm, row_half_mirror,
// row_mirror) within 16-lane rows and v_permlane16_swap / v_permlane32_swap
// across them.  The state broadcast for the right-hand side, per-reaction
// rates, the Jacobian assembly and the LU pivot row (v_readlane for whole-wave
// zones) go through a per-group LDS area.
//
// Methods (the kernel's fourth template parameter): the fixed-leading-
// coefficient BDF with a Jacobian every step or the Jacobian/LU reuse, the
// damped Runge-Kutta-Chebyshev method, and the variable-coefficient BDF with
// either Jacobian policy.
//
// Scheduling.  The grid is persistent: every group pulls the next zone from
// a device-wide atomic counter when its zone is done, so zones of very
// different cost share the machine until the queue is empty.  Several
// segments (networks) can share one launch when they use the same kernel.
//
// The integrator follows the rules of the CPU oracle (Nordsieck BDF, orders
// 1..5, Hairer-Norsett-Wanner start, Newton with kappa 0.03, biased order and
// step selection, failure statuses); see the header comment of include/zoneburn.h.

#pragma once

#include <float.h>
#include <math.h>

#include <type_traits>
#include <utility>

#include "zb_internal.h"
#include "zb_log.h"
#include "zb_stepmath.h"
#include "zoneburn.h"

namespace zb {

// ----------------------------------------------------------------- lane ops

// Orders one lane's LDS stores before other lanes' later LDS loads.  Every workgroup
// is a single wave, and the LDS performs one wave's accesses in issue order, so a
// wavefront-scope fence suffices: it keeps the compiler from moving LDS accesses
// across it and emits no wait for outstanding stores.
__device__ __forceinline__ void lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pivot reciprocal, off the IEEE division sequence, whose dependent chain each elimination
// step waits on.  FP64: the hardware approximation refined by two Newton steps (within about
// an ulp; on 2^20 zones of the 14-variable network every result came out bitwise as with the
// division).  FP32 (the mixed-precision LU, an approximate factorisation the Newton
// iteration absorbs): the hardware reciprocal alone, within an ulp.  A zero pivot still
// yields a non-finite factor and so a failed Newton iteration.
__device__ __forceinline__ double recip(double x) { return zbm::recip_from(x, __builtin_amdgcn_rcp(x)); }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Load from global memory.  The network tables reach the kernel through generic
// pointers, which compile to flat loads; those also count against the LDS wait counter,
// so every LDS wait would wait for them too.
typedef int zb_v4i __attribute__((ext_vector_type(4)));
typedef double zb_v2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int4 gload(const int4 *p)
{
    const zb_v4i v = *(const __attribute__((address_space(1))) zb_v4i *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double4 gload(const double4 *p)
{
    const __attribute__((address_space(1))) zb_v2d *q = (const __attribute__((address_space(1))) zb_v2d *)p;
    const zb_v2d a = q[0], b = q[1];
    return make_double4(a.x, a.y, b.x, b.y);
}

// Every DPP pattern used here (quad_perm, row_half_mirror, row_mirror, row_newbcast) reads a
// lane of the same 16-lane row, so no lane keeps its old value: the move takes no old operand
// (no extra instruction to set one).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    int lo = dpp_i<CTRL>((int)(u & 0xffffffffu));
    int hi = dpp_i<CTRL>((int)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}

template <int CTRL>
__device__ __forceinline__ int dpp(int v)
{
    return dpp_i<CTRL>(v);
}

// Marks a value as an opaque register so that a chain of selects over a
// register array is not rewritten into an indexed load (which would move the
// whole array to scratch memory).
__device__ __forceinline__ double opq(double v) { asm volatile("" : "+v"(v)); return v; }
__device__ __forceinline__ float opq(float v) { asm volatile("" : "+v"(v)); return v; }

// v, made to depend on d (no instruction).  Keeps the scheduler from computing
// the per-step owner masks of a triangular solve ahead of the dependent chain,
// which would hold one scalar mask per step live at once.
template <class D>
__device__ __forceinline__ int after(int v, D d) { asm volatile("" : "+v"(v) : "v"(d)); return v; }

// A wave-uniform integer made to depend on d (no instruction): bounds how far the
// scheduler can hoist scalar reads that use it.
template <class D>
__device__ __forceinline__ int after_s(int v, D d) { asm volatile("" : "+s"(v) : "v"(d)); return v; }

// A private copy of a wave-uniform integer (no instruction).  Comparisons of
// the LU and solve loops against the network size are then not shared between
// those routines, which would keep one scalar mask per column live across a
// whole step.
__device__ __forceinline__ int own_copy(int v) { asm volatile("" : "+s"(v)); return v; }

// Compile-time loop: f(std::integral_constant<int, i>) for i = B .. E-1.  Indices of
// register arrays stay constant expressions even where a loop bound depends on an
// outer index, which ordinary unrolling does not guarantee.
template <int B, class F, int... I>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, B + I>{}), ...);
}

template <int B, int E, class F>
__device__ __forceinline__ void sfor(F &&f)
{
    if constexpr (E > B) sfor_impl<B>(f, std::make_integer_sequence<int, E - B>{});
}

struct OpAdd { template <class T> __device__ T operator()(T a, T b) const { return a + b; } };
// max and min of floating values as single v_max / v_min instructions (the same result as a
// compare and select for every non-NaN value)
struct OpMax {
    template <class T> __device__ T operator()(T a, T b) const
    {
        if constexpr (std::is_floating_point_v<T>) return fmax(a, b); else return a > b ? a : b;
    }
};
struct OpMin {
    template <class T> __device__ T operator()(T a, T b) const
    {
        if constexpr (std::is_floating_point_v<T>) return fmin(a, b); else return a < b ? a : b;
    }
};

// Exchange across 16-lane rows without LDS (gfx950 v_permlane16_swap /
// v_permlane32_swap).  Swapping a register with itself leaves, in the pair
// (r0, r1), this lane's value and that of the lane 16 (32) positions away, in an
// order that depends on the row; a commutative op of the two is the same in both
// partner lanes.
template <int D>
__device__ __forceinline__ void xswap(unsigned v, unsigned &a, unsigned &b)
{
    if constexpr (D == 16) {
        auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        a = r[0];
        b = r[1];
    } else {
        auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        a = r[0];
        b = r[1];
    }
}

template <int D, class Op>
__device__ __forceinline__ double xrow(double v, Op op)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    unsigned a0, b0, a1, b1;
    xswap<D>((unsigned)(u & 0xffffffffu), a0, b0);
    xswap<D>((unsigned)(u >> 32), a1, b1);
    double x = __longlong_as_double((long long)(((unsigned long long)a1 << 32) | a0));
    double y = __longlong_as_double((long long)(((unsigned long long)b1 << 32) | b0));
    return op(x, y);
}

template <int D, class Op>
__device__ __forceinline__ float xrow(float v, Op op)
{
    unsigned a, b;
    xswap<D>(__float_as_uint(v), a, b);
    return op(__uint_as_float(a), __uint_as_float(b));
}

template <int D, class Op>
__device__ __forceinline__ int xrow(int v, Op op)
{
    unsigned a, b;
    xswap<D>((unsigned)v, a, b);
    return op((int)a, (int)b);
}

// All-reduce over the L lanes of a group; every lane receives the same bits
// (the ops are commutative, and every stage combines the same pair in both lanes).
template <int L, class T, class Op>
__device__ __forceinline__ T greduce(T v, Op op)
{
    if constexpr (L >= 2) v = op(v, dpp<0xB1>(v));     // quad_perm [1,0,3,2]
    if constexpr (L >= 4) v = op(v, dpp<0x4E>(v));     // quad_perm [2,3,0,1]
    if constexpr (L >= 8) v = op(v, dpp<0x141>(v));    // row_half_mirror
    if constexpr (L >= 16) v = op(v, dpp<0x140>(v));   // row_mirror
    if constexpr (L >= 32) v = xrow<16>(v, op);
    if constexpr (L >= 64) v = xrow<32>(v, op);
    return v;
}

// Whole-wave groups: the value of the lowest lane whose flag is set, in every
// lane (zero when no lane is flagged), read with v_readlane.
template <class T>
__device__ __forceinline__ T wave_pick(T v, bool flag)
{
    unsigned long long m = __ballot(flag);
    if (m == 0ull) return T(0);
    const int src = __builtin_ctzll(m);
    if constexpr (sizeof(T) == 8) {
        unsigned long long u = (unsigned long long)__double_as_longlong(v);
        unsigned lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffu), src);
        unsigned hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
    }
}

// Value of lane K of the group (K a constant), in every lane of the group, without LDS:
// quad_perm for L <= 4, row_newbcast (gfx90a+) within 16-lane rows, a permlane16 swap
// between the two rows of a 32-lane group, v_readlane for a whole wave.
template <int L, int K>
__device__ __forceinline__ unsigned bcast_k32(unsigned v)
{
    static_assert(K >= 0 && K < L, "lane out of the group");
    if constexpr (L == 1) {
        return v;
    } else if constexpr (L == 2) {
        return (unsigned)dpp_i<K | (K << 2) | ((2 + K) << 4) | ((2 + K) << 6)>((int)v);
    } else if constexpr (L == 4) {
        return (unsigned)dpp_i<K | (K << 2) | (K << 4) | (K << 6)>((int)v);
    } else if constexpr (L == 8) {
        unsigned a = (unsigned)dpp_i<0x150 + K>((int)v), b = (unsigned)dpp_i<0x158 + K>((int)v);
        return (threadIdx.x & 8) ? b : a;
    } else if constexpr (L == 16) {
        return (unsigned)dpp_i<0x150 + K>((int)v);
    } else if constexpr (L == 32) {
        unsigned a = (unsigned)dpp_i<0x150 + (K & 15)>((int)v), r0, r1;
        xswap<16>(a, r0, r1);   // r0: the even row's value, r1: the odd row's, in both rows
        return K < 16 ? r0 : r1;
    } else {
        return (unsigned)__builtin_amdgcn_readlane((int)v, K);
    }
}

template <int L, int K>
__device__ __forceinline__ double bcast_k(double v)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    unsigned lo = bcast_k32<L, K>((unsigned)(u & 0xffffffffu));
    unsigned hi = bcast_k32<L, K>((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int L, int K>
__device__ __forceinline__ float bcast_k(float v)
{
    return __uint_as_float(bcast_k32<L, K>(__float_as_uint(v)));
}

// Value of lane src (wave-uniform) of the wave, with v_readlane.
__device__ __forceinline__ double lane_read(double v, int src)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffu), src);
    unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), src);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ float lane_read(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Value of lane src of the wave (ds_bpermute; no LDS memory is touched).
__device__ __forceinline__ double gather(double v, int src)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)(u & 0xffffffffu));
    unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ float gather(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// Value held by the single owner lane of the group, delivered to every lane.
template <int L, class T>
__device__ __forceinline__ T gbcast(T v, bool owner)
{
    if constexpr (L == 64) return wave_pick(v, owner);
    else return greduce<L>(owner ? v : T(0), OpAdd());
}


// A group-uniform flag, stated as such for whole-wave groups (so code under it may keep
// wave-uniform values in scalar registers).
template <int L>
__device__ __forceinline__ bool group_uniform(bool b)
{
    if constexpr (L == 64) return __builtin_amdgcn_readfirstlane((int)b) != 0;
    else return b;
}

template <int L>
__device__ __forceinline__ bool gany(bool b)
{
    return greduce<L>(b ? 1 : 0, OpMax()) != 0;
}

// Integration methods (the compile-time fourth parameter of the burn kernel): the
// fixed-leading-coefficient BDF with a Jacobian every step or reused, RKC, and the
// variable-coefficient BDF with either Jacobian policy.
constexpr int RKC_SMAX = 250;

// ------------------------------------------------------------- step control
// The WRMS norms and the step-size factors start from the hardware approximations
// (v_rcp_f64, v_sqrt_f64, the FP32 log2 and exp2) and are refined by Newton steps to about
// 1 ulp, so the step sizes and accept/reject decisions agree with the exact formulas as
// closely as the library routines would: about 15 instructions for a norm against ~36 for
// a division and a correctly rounded square root, about 50 for a factor against ~180 for a
// pow and a division.

// Root mean square from a sum of n squares (0, +inf and NaN keep their meaning).
__device__ __forceinline__ double rms_of_sum(double s, int n)
{
    const double dn = (double)n;
    const double x = s * zbm::recip_from(dn, __builtin_amdgcn_rcp(dn));
    const double y0 = __builtin_amdgcn_sqrt(x);
    const double y = zbm::sqrt_from(x, y0, __builtin_amdgcn_rcp(y0));
    return (x > 0.0 && x < __builtin_inf()) ? y : y0;
}

// x^(1/k) for x >= 0 (or NaN) and 1 <= k <= 6, as pow(x, 1/k) gives it.  x = 2^(k j) xs
// with j from the exponent of x, so that xs lies within a few powers of two of 1 and the
// FP32 start is in range for every positive double; the root is 2^j xs^(1/k), the scalings
// exact.
__device__ __forceinline__ double kth_root(double x, int k)
{
    const float rk = __builtin_amdgcn_rcpf((float)k);
    const int j = (int)((float)__builtin_amdgcn_frexp_exp(x) * rk);
    const double xs = __builtin_amdgcn_ldexp(x, -k * j);
    const double y0 = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)xs) * rk);
    const double y = __builtin_amdgcn_ldexp(
        zbm::root_from(xs, k, y0, [](double d) { return __builtin_amdgcn_rcp(d); }), j);
    return (x > 0.0 && x < __builtin_inf()) ? y : x;   // 0, +inf and NaN pass through
}

// Step-size factor 1 / (x^(1/k) + 1e-6) of the error and order tests, x = b E >= 0.
__device__ __forceinline__ double step_factor(double x, int k)
{
    const double d = kth_root(x, k) + 1e-6;
    return (d < __builtin_inf()) ? zbm::recip_from(d, __builtin_amdgcn_rcp(d)) : 1.0 / d;
}

// --------------------------------------------------------- BDF coefficients

// l_j(q): coefficients of prod_{i<=q} (1 + x/i) divided by H_q (so l_1 = 1).
__device__ __forceinline__ double lcoef(int q, int j)
{
    // rows q = 1..5, columns j = 0..5, exact rationals rounded once
    const double t[5][6] = {
        {1.0, 1.0, 0.0, 0.0, 0.0, 0.0},
        {2.0 / 3.0, 1.0, 1.0 / 3.0, 0.0, 0.0, 0.0},
        {6.0 / 11.0, 1.0, 6.0 / 11.0, 1.0 / 11.0, 0.0, 0.0},
        {12.0 / 25.0, 1.0, 7.0 / 10.0, 1.0 / 5.0, 1.0 / 50.0, 0.0},
        {60.0 / 137.0, 1.0, 225.0 / 274.0, 85.0 / 274.0, 15.0 / 274.0, 1.0 / 274.0}};
    double v = t[0][j];
#pragma unroll
    for (int r = 1; r < 5; ++r)
        if (q == r + 1) v = t[r][j];
    return v;
}

// l_0(q) = 1 / H_q (the divisions are done by the compiler)
__device__ __forceinline__ double inv_harmonic(int q)
{
    double v = 1.0;
    v = (q == 2) ? 1.0 / 1.5 : v;
    v = (q == 3) ? 1.0 / (11.0 / 6.0) : v;
    v = (q == 4) ? 1.0 / (25.0 / 12.0) : v;
    v = (q == 5) ? 1.0 / (137.0 / 60.0) : v;
    return v;
}

// H_q = 1 / l_0(q)
__device__ __forceinline__ double harmonic(int q)
{
    double v = 1.0;
    v = (q == 2) ? 1.5 : v;
    v = (q == 3) ? 11.0 / 6.0 : v;
    v = (q == 4) ? 25.0 / 12.0 : v;
    v = (q == 5) ? 137.0 / 60.0 : v;
    return v;
}

// c(n, j) = [x^j] x (x+1) ... (x+n-1), n = 2..6
__device__ __forceinline__ double stirling(int n, int j)
{
    const double t[5][7] = {
        {0, 1, 1, 0, 0, 0, 0},
        {0, 2, 3, 1, 0, 0, 0},
        {0, 6, 11, 6, 1, 0, 0},
        {0, 24, 50, 35, 10, 1, 0},
        {0, 120, 274, 225, 85, 15, 1}};
    double v = t[0][j];
#pragma unroll
    for (int r = 1; r < 5; ++r)
        if (n == r + 2) v = t[r][j];
    return v;
}

// (2/3 - 1e-6)^n for n = 1..6
__device__ __forceinline__ double cpow23(int n)
{
    const double c = 2.0 / 3.0 - 1e-6;
    double v = c;
    v = (n >= 2) ? v * c : v;
    v = (n >= 3) ? v * c : v;
    v = (n >= 4) ? v * c : v;
    v = (n >= 5) ? v * c : v;
    v = (n >= 6) ? v * c : v;
    return v;
}

__device__ __forceinline__ double factorial(int n)
{
    double v = 1.0;
    v = (n == 2) ? 2.0 : v;
    v = (n == 3) ? 6.0 : v;
    v = (n == 4) ? 24.0 : v;
    v = (n == 5) ? 120.0 : v;
    v = (n == 6) ? 720.0 : v;
    return v;
}

// ------------------------------------------------------------- zone state

template <int NVP, int L, class LT>
struct Zone {
    static constexpr int RPL = (NVP + L - 1) / L;
    double Z[QMAX + 1][RPL];    // Nordsieck history, local rows (the copy taken before
                                // each prediction is kept in LDS, or in registers of the
                                // attempt where hist_regs says so)
    double dyp[RPL];            // dy of the previous accepted step
    double iw[RPL];             // 1 / (atol + rtol |y|)
    double y[RPL], dy[RPL], f[RPL];
    double src[RPL];            // constant source of the zone (0 without one)
    double rtol, atol;          // tolerances of the current run (the retry may loosen them)
    int max_steps, tries;
    int fdj;                    // Jacobian by finite differences (a retry option)
    // iteration-matrix state for the VODE-style reuse (jac_policy 1)
    double gamma_m;             // gamma the factors in M were formed with
    double cs[RPL];             // column scale of the factors (mixed: the error weight then)
    int have_j, have_m, nst_j, nst_m;
    LT M[RPL][NVP];             // iteration matrix rows, then their LU factors
    LT dinv[RPL];               // 1 / pivot of the row (valid once it is a pivot row)
    LT rs[RPL];                 // row scaling of the FP32 LU
    int pstep[RPL];             // elimination step at which the row was the pivot
    int pivlane;                // one row per lane: group lane whose row is pivot row gl
                                // (the rows are moved there once the LU is complete)
    double t, h;
    int q, nequal, nefc, ncfc;
    int nst, nfe, nje, nlu, nni, netf, ncf;
};

// Lane context: the group's identity, its LDS area and the zone's network.
struct Ctx {
    int gl;                  // lane within the group
    double *S;               // group LDS base
    LdsLayout lay;
    int seg;                 // the segment worked on (wave-uniform)
    int ns, nv;              // its network's species and integrated variables
    int64_t zone;
    int jac_policy;
    bool lu_blocked;         // the blocked matrix-core LU (48-row FP32 kernels)
    bool rates;              // per-reaction rate factors in LDS (else all 1)
};

template <int NVP, int L>
__device__ __forceinline__ int row_of(const Ctx &c, int s) { return c.gl + L * s; }

// The segment's network tables and buffers, read from the kernel-argument segment where
// they are used.  Held in scalar registers through the persistent loop, they (with the
// loop's other uniform values) overflowed the scalar register file and were spilled to
// lanes of vector registers, each reload of the 16-register block costing 16 vector
// instructions.  The loads hit the scalar cache; the opaque segment index keeps the
// compiler from hoisting them out of the loop again.
__device__ __forceinline__ const Segment &seg_of(const Ctx &c)
{
    const BurnArgs *pa = (const BurnArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    return pa->seg[own_copy(c.seg)];
}

__device__ __forceinline__ DevNet net_of(const Ctx &c)
{
    const DevNet &n = seg_of(c).net;
    DevNet r;
    r.ns = c.ns;
    r.nv = c.nv;
    r.thermal = n.thermal;
    r.nr = n.nr;
    r.inv_len = n.inv_len;
    r.rct = n.rct;
    r.par = n.par;
    r.inv = n.inv;
    return r;
}

// Per-reaction rate factors in LDS, used when the launch has any (rate scales, or the constant
// rates of a network without temperature); otherwise they are all 1 and neither written nor
// read (the trimmed layout has no room for them then).
template <int NVP, int L, class LT>
__device__ __forceinline__ bool rates_in_lds(const Ctx &c)
{
    return c.rates;
}

// Element type of the Jacobian rows in LDS.
template <int NVP, class LT>
using JacT = std::conditional_t<jac_f32(NVP, sizeof(LT) == 4), float, double>;

// Weighted RMS norm over the nv integrated components.
template <int NVP, int L, class LT>
__device__ __forceinline__ double wrms(const Ctx &c, const Zone<NVP, L, LT> &z,
                                       const double (&v)[Zone<NVP, L, LT>::RPL])
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        if (row_of<NVP, L>(c, k) < c.nv) {
            double x = v[k] * z.iw[k];
            s = fma(x, x, s);
        }
    }
    s = greduce<L>(s, OpAdd());
    return rms_of_sum(s, c.nv);
}

// ------------------------------------------------------------- network

// f(y) for the group's zone; with WANTJ also assembles M = I - gamma J (and
// its FP32 scaling) in registers.  y and f are by local row.
template <bool WANTJ, int NVP, int L, class LT>
__device__ __forceinline__ void eval(const Ctx &c, Zone<NVP, L, LT> &z, const double (&yv)[Zone<NVP, L, LT>::RPL],
                     double (&fo)[Zone<NVP, L, LT>::RPL])
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    const DevNet N = net_of(c);
    double *ybuf = c.S + c.lay.ybuf;
    double *ks = c.S + c.lay.ks;
    double *rx = c.S + c.lay.rx;
    using JT = JacT<NVP, LT>;
    JT *jb = (JT *)(c.S + c.lay.jbuf);

    // The 14-row kernels with a Jacobian every step (one row a lane, registers to spare): a
    // row's whole list, up to 6 entry pairs, is loaded first, so its latency overlaps the
    // rate evaluation, and walked from registers.  Elsewhere the extra registers cost
    // occupancy or spills, and the list is streamed.
    constexpr int PMAX = (RPL == 1 && NVP == 14 && L == 16) ? 6 : 0;
    int4 pre[PMAX > 0 ? PMAX : 1];
    const int n2 = N.inv_len / 2;
    const bool use_pre = PMAX > 0 && c.jac_policy == 0 && n2 <= PMAX;
    if constexpr (PMAX > 0) {
        const int i0 = row_of<NVP, L>(c, 0);
        const int4 *l0 = (const int4 *)(N.inv + (i0 < N.ns ? i0 : 0) * N.inv_len);
        sfor<0, PMAX>([&](auto P) {
            pre[P] = make_int4(0, 0, 0, 0);
            if (use_pre && P < n2) pre[P] = gload(l0 + P);
        });
    }
    // one row a lane: T from its lane through the LDS crossbar, so that its logarithm and
    // reciprocal overlap the stores below instead of waiting for them
    double Tg = 0.0;
    if constexpr (RPL == 1) Tg = gather(yv[0], (int)(threadIdx.x & (64 - L)) + N.ns);
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        int i = row_of<NVP, L>(c, s);
        if (i < N.nv) ybuf[i] = yv[s];
    }
    double lnT = 0.0, iT = 0.0;
    if constexpr (RPL == 1) {
        if (N.thermal) {
            lnT = zbm::log_series(Tg);
            iT = zbm::recip_from(Tg, __builtin_amdgcn_rcp(Tg));
        }
    }
    constexpr int JS = NVP + 1;   // Jacobian row stride in LDS
    const int nr = N.nr;
    if (WANTJ) {
        // clear the Jacobian rows this lane owns (the row walk below adds into them) and its
        // species' entries of the T row (the reactions add into those; the T row's T entry is
        // written whole)
        sfor<0, RPL>([&](auto S) {
            int i = row_of<NVP, L>(c, S);
            if (i < N.ns) {
                sfor<0, NVP>([&](auto J) { jb[i * JS + J] = JT(0); });
                jb[N.ns * JS + i] = JT(0);
            }
        });
    }
    lds_fence();

    if (RPL > 1 && N.thermal) {
        double T = ybuf[N.ns];
        lnT = zbm::log_series(T);
        // the hardware reciprocal refined (zb_stepmath.h): on 2^20 zones of the 14-variable
        // network the results came out bitwise as with the division, at fewer instructions
        iT = zbm::recip_from(T, __builtin_amdgcn_rcp(T));
    }
    double sT = 0.0, sTT = 0.0;
    // the next reaction's parameters are loaded while the current one is processed
    int4 nix = make_int4(0, -1, 0, 0);
    double4 npr = make_double4(0.0, 0.0, 0.0, 0.0);
    if (c.gl < N.nr) {
        nix = gload(N.rct + c.gl);
        npr = gload(N.par + c.gl);
    }
    for (int r = c.gl; r < N.nr; r += L) {
        const int4 ix = nix;
        const double4 pr = npr;
        if (r + L < N.nr) {
            nix = gload(N.rct + r + L);
            npr = gload(N.par + r + L);
        }
        // sign-aware mass action: w = s k Ya Yb with s = -1 when both reactants are
        // negative (k Ya |Ya| for A + A), so a negative abundance is pulled back to 0
        const double ya = ybuf[ix.x];
        const double yb0 = ix.y >= 0 ? ybuf[ix.y] : 1.0;
        const double yb = (ya < 0.0 && yb0 < 0.0) ? -yb0 : yb0;
        double k = rates_in_lds<NVP, L, LT>(c) ? ks[r] : 1.0;
        if (N.thermal) k *= exp(pr.x + pr.y * lnT - pr.z * iT);
        double kYb = k * yb;
        double w = kYb * ya;
        rx[r] = w;
        if (WANTJ) {
            double kb = ix.y >= 0 ? ((ya < 0.0 && yb0 < 0.0) ? -k * ya : k * ya) : 0.0;
            double kt = N.thermal ? w * (pr.y + pr.z * iT) * iT : 0.0;
            rx[nr + r] = kYb;
            rx[2 * nr + r] = kb;
            rx[3 * nr + r] = kt;
            sTT += pr.w * kt;
            if (N.thermal) {
                // T row: q_r dw_r/dY for each reactant of the reaction, added in place, so
                // that no lane walks a list of the reactions its species is consumed by
                // (a chain of dependent table loads: 8 % of the burn on the 14-variable network)
                JT *trow = jb + N.ns * JS;
                __hip_atomic_fetch_add(trow + ix.x, (JT)(pr.w * kYb), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                if (ix.y >= 0)
                    __hip_atomic_fetch_add(trow + ix.y, (JT)(pr.w * kb), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        sT += pr.w * w;
    }
    double fT = 0.0, JTT = 0.0;
    if (N.thermal) {
        fT = greduce<L>(sT, OpAdd());
        if (WANTJ) JTT = greduce<L>(sTT, OpAdd());
    }
    lds_fence();

#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        int i = row_of<NVP, L>(c, s);
        double fi = 0.0;
        if (i < N.ns) {
            // two list entries per iteration (one 16-byte load), contributions added
            // in list order; each entry carries the reactant columns it feeds
            const int4 *lst = (const int4 *)(N.inv + i * N.inv_len);
            double jit = 0.0;
            JT *jrow = jb + i * JS;
            auto jadd = [&](int y, double nu, double da, double db) {
                const int a = y & 0xff, b = (y >> 8) - 1;
                __hip_atomic_fetch_add(jrow + a, (JT)(nu * da), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                if (b >= 0)
                    __hip_atomic_fetch_add(jrow + b, (JT)(nu * db), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            };
            // A pair of entries: the second is taken under a predicate (a padding entry
            // reads slot 0 and adds nothing), so the LDS reads of both go out together.
            auto pair = [&](int4 en) {
                const int n0 = en.x >> 16, n1 = en.z >> 16;   // nu; 0 on a padding entry
                const bool has1 = n1 != 0;
                const int r0 = en.x & 0xffff, r1 = has1 ? (en.z & 0xffff) : 0;
                const double nu0 = (double)n0;
                const double nu1 = (double)n1;
                const double w0 = rx[r0], w1 = rx[r1];
                double p0 = 0.0, p1 = 0.0, q0 = 0.0, q1 = 0.0, t0 = 0.0, t1 = 0.0;
                if (WANTJ) {
                    p0 = rx[nr + r0]; p1 = rx[nr + r1];
                    q0 = rx[2 * nr + r0]; q1 = rx[2 * nr + r1];
                    t0 = rx[3 * nr + r0]; t1 = rx[3 * nr + r1];
                }
                fi = fma(nu0, w0, fi);
                if (has1) fi = fma(nu1, w1, fi);
                if (WANTJ) {
                    jadd(en.y, nu0, p0, q0);
                    jit = fma(nu0, t0, jit);
                    if (has1) {
                        jadd(en.w, nu1, p1, q1);
                        jit = fma(nu1, t1, jit);
                    }
                }
            };
            if (use_pre) {
                // entries past the row's list are padding (nu = 0), skipped
                sfor<0, (PMAX > 0 ? PMAX : 1)>([&](auto P) {
                    if (P < n2 && (pre[P].x >> 16) != 0) pair(pre[P]);
                });
            } else {
                int4 nen = n2 > 0 ? gload(lst) : make_int4(0, 0, 0, 0);
                for (int e = 0; e < n2; ++e) {
                    const int4 en = nen;
                    if (e + 1 < n2) nen = gload(lst + e + 1);
                    if ((en.x >> 16) == 0) break;
                    pair(en);
                    if ((en.z >> 16) == 0) break;
                }
            }
            if (WANTJ && N.thermal) jrow[N.ns] = (JT)jit;
        } else if (N.thermal && i == N.ns) {
            fi = fT;
            if (WANTJ) jb[N.ns * JS + N.ns] = (JT)JTT;
        }
        fo[s] = fi + z.src[s];
    }

}

// Forward-difference Jacobian at y, the alternative Jacobian approximation of a
// zone-by-zone retry: column j = (f(y + d_j e_j) - f(y)) / d_j with
// d_j = 2^-26 max(|y_j|, atol + rtol |y_j|) replaced by (y_j + d_j) - y_j, so that it is
// exactly the change applied.  Leaves f(y) in fo and the rows where eval<true> leaves
// them; the nv perturbed evaluations are counted in nfe.
template <int NVP, int L, class LT>
__device__ __forceinline__ void fd_jacobian(const Ctx &c, Zone<NVP, L, LT> &z,
                                            const double (&yv)[Zone<NVP, L, LT>::RPL],
                                            double (&fo)[Zone<NVP, L, LT>::RPL])
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    constexpr int JS = NVP + 1;
    using JT = JacT<NVP, LT>;
    JT *jb = (JT *)(c.S + c.lay.jbuf);
    eval<false>(c, z, yv, fo);
    const int nv = c.nv;
    for (int j = 0; j < nv; ++j) {
        double yp[RPL], fp[RPL];
        double dj = 0.0;
        bool own = false;
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            const double y = yv[s];
            yp[s] = y;
            if (row_of<NVP, L>(c, s) == j) {
                const double d = 0x1p-26 * fmax(fabs(y), z.atol + z.rtol * fabs(y));
                yp[s] = y + d;
                dj = yp[s] - y;
                own = true;
            }
        }
        dj = gbcast<L>(dj, own);
        eval<false>(c, z, yp, fp);
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            const int i = row_of<NVP, L>(c, s);
            if (i < nv) jb[i * JS + j] = (JT)((fp[s] - fo[s]) / dj);
        }
        z.nfe++;
    }
}

// M = I - gamma J from the Jacobian rows in LDS (left there by eval<true>), in
// registers.  The mixed path scales column j by the error weight w_j and the row by
// 1 / max; the column scales in force are kept per zone for the solves, since a matrix
// may be reused at later steps.
// Kernels with one row a lane factor with the pivot order of the zone's previous
// factorisation kept while it stays acceptable (lu_kept_order); the blocked matrix-core LU
// does its own pivoting from the natural order.
template <int NVP, int L, class LT>
constexpr bool kept_order() { return Zone<NVP, L, LT>::RPL == 1 && L >= 2; }

template <int NVP, int L, class LT>
__device__ __forceinline__ void form_M(const Ctx &c, Zone<NVP, L, LT> &z, double gamma)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    constexpr int JS = NVP + 1;
    const DevNet N = net_of(c);
    const JacT<NVP, LT> *jb = (const JacT<NVP, LT> *)(c.S + c.lay.jbuf);
    lds_fence();
    constexpr bool MIXED = sizeof(LT) == 4;
    const double *wb = c.S + c.lay.wbuf;
    sfor<0, RPL>([&](auto S) {
        // one row a lane: the lane forms the row it held after the zone's last factorisation
        // (the pivot order, identity at the zone's start); else its own rows
        int i = (kept_order<NVP, L, LT>() && !c.lu_blocked) ? z.pivlane : row_of<NVP, L>(c, S);
        double rmax = 0.0;
        double mrow[NVP];
        if (i < N.nv) {
            sfor<0, NVP>([&](auto J) {
                double m = (J == i ? 1.0 : 0.0) - gamma * (double)jb[i * JS + J];
                if (J >= N.nv) m = (J == i) ? 1.0 : 0.0;
                if (MIXED) {
                    m *= wb[J];
                    rmax = fmax(rmax, fabs(m));
                }
                mrow[J] = m;
            });
        } else {
            sfor<0, NVP>([&](auto J) { mrow[J] = (J == i) ? 1.0 : 0.0; });
            rmax = 1.0;
        }
        if (MIXED) {
            double sc = rmax > 0.0 ? zbm::recip_from(rmax, __builtin_amdgcn_rcp(rmax)) : 1.0;
            z.rs[S] = (LT)sc;
            sfor<0, NVP>([&](auto J) { z.M[S][J] = (LT)(mrow[J] * sc); });
        } else {
            sfor<0, NVP>([&](auto J) { z.M[S][J] = (LT)mrow[J]; });
        }
    });
    sfor<0, RPL>([&](auto S) {
        const int i = row_of<NVP, L>(c, S);
        z.cs[S] = (i < NVP) ? c.S[c.lay.wbuf + i] : 1.0;
    });
}

// --------------------------------------------------------------- LU / solve

// Runs f(k) for the elimination steps k of nv variables, testing nv once per 8 steps instead
// of per step, so that 8 steps form one block the scheduler can overlap.  Steps past nv up to
// the next multiple of 8 (and nvp) run too; they are harmless in the LU and the solves: the
// rows of M past nv are identity rows (pivot 1, every other multiplier 0) and the right-hand
// side is zero there.  REV runs the steps backwards (nvp-1 first).
template <int NVP, bool REV = false, class F>
__device__ __forceinline__ void steps8(int nv, F &&f)
{
    sfor<0, (NVP + 7) / 8>([&](auto C) {
        constexpr int a = 8 * C, b = (8 * C + 8 < NVP) ? 8 * C + 8 : NVP;
        if constexpr (!REV) {
            if (a < nv) sfor<a, b>(f);
        } else {
            // chunk C holds k = NVP-1-kk for kk in [a, b)
            if (NVP - b < nv)
                sfor<a, b>([&](auto KK) { f(std::integral_constant<int, NVP - 1 - KK>{}); });
        }
    });
}

typedef float zb_v16f __attribute__((ext_vector_type(16)));
typedef float zb_v4f __attribute__((ext_vector_type(4)));

// The LU of the whole-wave 48-row FP32 kernels, blocked for the matrix cores, under the
// every-step Jacobian policy.  Three panels of 16 columns.  A panel is factored as in the
// unblocked code (pivot search, multipliers, rank-1 updates), the updates kept to the
// panel's own columns.  The columns right of it then take the panel's updates at once:
//  - the panel's pivot rows are reduced by the panel's unit lower triangle (a 16-step
//    triangular solve, one column per lane), giving U, their final parts there;
//  - the rows still unpivoted (32 after the first panel, 16 after the second, in lane
//    order) lose Lp U, Lp their multipliers of the panel: one product on the matrix cores,
//    v_mfma_f32_32x32x2f32 for 32 x 32 x 16, v_mfma_f32_16x16x4f32 for 16 x 16 x 16.
// Operands and product change lane layout through the Jacobian's LDS area, which is unused
// from the formation of M to the next Jacobian.  Rows of M past nv are identity rows and
// come last in lane order, so every row with a nonzero update fits the product.
template <int NVP, int L, class LT>
__device__ __forceinline__ void lu_factor_blocked(const Ctx &c, Zone<NVP, L, LT> &z)
{
    static_assert(NVP == 48 && L == 64 && sizeof(LT) == 4, "whole-wave 48-row FP32 LU");
    constexpr int PB = 16;                            // panel width
    constexpr int SU = 36, SA = 20, SL = 20, SD = 40; // LDS row strides (floats)
    float *const UT = (float *)(c.S + c.lay.jbuf);    // 16 x SU: pivot rows right of the panel
    float *const AT = UT + PB * SU;                    // 32 x SA: multipliers of unpivoted rows
    float *const LW = AT + 32 * SA;                    // 16 x SL: the panel's lower triangle
    float *const DT = AT;                              // 32 x SD: the product (AT, LW read by then)
    const int nv = own_copy(c.nv);
    const int lane = c.gl;
    z.pstep[0] = 127;
    z.pivlane = lane;
    sfor<0, NVP / PB>([&](auto P) {
        constexpr int c0 = P * PB;
        // nv is tested once per 8 steps, as in lu_factor (steps past nv pivot identity rows)
        auto elim = [&](auto KK) {
            constexpr int k = c0 + KK;
            LT bv = LT(-1);
            int bi = 1 << 20;
            {
                const LT a = fabs(z.M[0][k]);
                if (z.pstep[0] > k && lane < NVP && a > bv) {
                    bv = a;
                    bi = lane;
                }
            }
            const LT gm = greduce<L>(bv, OpMax());
            const unsigned long long msk = __ballot(bv == gm && bi < (1 << 20));
            const int p = msk ? (int)__builtin_ctzll(msk) : (1 << 20);
            const LT rinv = recip(lane_read(z.M[0][k], p));
            if (lane == p) {
                z.pstep[0] = k;
                z.dinv[0] = rinv;
            }
            const bool act = z.pstep[0] > k;
            const LT l = act ? z.M[0][k] * rinv : LT(0);
            if (act) z.M[0][k] = l;
            int pp = p;
            sfor<k + 1, c0 + PB>([&](auto J) {
                if constexpr (J % 8 == 0) pp = after_s(pp, z.M[0][J - 1]);
                z.M[0][J] = fma(-l, lane_read(z.M[0][J], pp), z.M[0][J]);
            });
            if (lane == k) z.pivlane = p;
        };
        sfor<0, PB / 8>([&](auto H) {
            if (c0 + 8 * H < nv) sfor<8 * H, 8 * H + 8>(elim);
        });
        if constexpr (c0 + PB < NVP) {
            constexpr int NT = NVP - c0 - PB;         // columns right of the panel = rows left
            const bool unp = lane < NVP && z.pstep[0] >= c0 + PB;
            const unsigned long long um = __ballot(unp);
            const int ci = (int)__builtin_amdgcn_mbcnt_hi(
                (unsigned)(um >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)um, 0u));
            const int kk = z.pstep[0] - c0;
            const bool piv = lane < NVP && kk >= 0 && kk < PB;
            const bool inA = unp && ci < NT;
            lds_fence();
            if (inA) {
                float a[PB];
                sfor<0, PB>([&](auto KK) { a[KK] = (c0 + KK < nv) ? z.M[0][c0 + KK] : 0.0f; });
                float4 *ar = (float4 *)(AT + ci * SA);
                if constexpr (P == 0) {   // [k % 2][k / 2]: the 32x32x2 A layout
                    ar[0] = make_float4(a[0], a[2], a[4], a[6]);
                    ar[1] = make_float4(a[8], a[10], a[12], a[14]);
                    ar[2] = make_float4(a[1], a[3], a[5], a[7]);
                    ar[3] = make_float4(a[9], a[11], a[13], a[15]);
                } else {                  // [k % 4][k / 4]: the 16x16x4 A layout
                    ar[0] = make_float4(a[0], a[4], a[8], a[12]);
                    ar[1] = make_float4(a[1], a[5], a[9], a[13]);
                    ar[2] = make_float4(a[2], a[6], a[10], a[14]);
                    ar[3] = make_float4(a[3], a[7], a[11], a[15]);
                }
            }
            if (piv) {
                float4 *lr = (float4 *)(LW + kk * SL);
                sfor<0, PB / 4>([&](auto Q) {
                    constexpr int j = c0 + 4 * Q;
                    lr[Q] = make_float4(z.M[0][j], z.M[0][j + 1], z.M[0][j + 2], z.M[0][j + 3]);
                });
                float4 *ur = (float4 *)(UT + kk * SU);
                sfor<0, NT / 4>([&](auto Q) {
                    constexpr int j = c0 + PB + 4 * Q;
                    ur[Q] = make_float4(z.M[0][j], z.M[0][j + 1], z.M[0][j + 2], z.M[0][j + 3]);
                });
            }
            lds_fence();
            // U by columns, written back in place
            if (lane < NT) {
                float u[PB];
                sfor<0, PB>([&](auto KK) { u[KK] = (c0 + KK < nv) ? UT[KK * SU + lane] : 0.0f; });
                sfor<1, PB>([&](auto KK) {
                    constexpr int kq = KK;
                    if (c0 + kq >= nv) return;
                    const float *lr = LW + kq * SL;   // same address in every lane
                    sfor<0, kq>([&](auto JJ) { u[kq] = fma(-lr[JJ], u[JJ], u[kq]); });
                });
                sfor<0, PB>([&](auto KK) { UT[KK * SU + lane] = u[KK]; });
            }
            lds_fence();
            // Lp U for the unpivoted rows
            if constexpr (P == 0) {
                const int n = lane & 31, h = lane >> 5;
                const float4 x0 = *(const float4 *)(AT + n * SA + 8 * h);
                const float4 x1 = *(const float4 *)(AT + n * SA + 8 * h + 4);
                const float av[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                zb_v16f acc = {};
                sfor<0, PB / 2>([&](auto KB) {
                    constexpr int kb = KB;
                    const int r = 2 * kb + h;
                    const float b = (c0 + r < nv) ? UT[r * SU + n] : 0.0f;
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[kb], b, acc, 0, 0, 0);
                });
                lds_fence();
                sfor<0, 16>([&](auto V) {
                    constexpr int v = V;
                    DT[(8 * (v / 4) + 4 * h + (v % 4)) * SD + n] = acc[v];
                });
            } else {
                const int m = lane & 15, g = lane >> 4;
                const float4 x = *(const float4 *)(AT + m * SA + 4 * g);
                const float av[4] = {x.x, x.y, x.z, x.w};
                zb_v4f acc = {};
                sfor<0, PB / 4>([&](auto KB) {
                    constexpr int kb = KB;
                    const int r = 4 * kb + g;
                    const float b = (c0 + r < nv) ? UT[r * SU + m] : 0.0f;
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kb], b, acc, 0, 0, 0);
                });
                lds_fence();
                sfor<0, 4>([&](auto V) {
                    constexpr int v = V;
                    DT[(4 * g + v) * SD + m] = acc[v];
                });
            }
            lds_fence();
            // pivot rows take U, unpivoted rows lose Lp U
            if (inA || piv) {
                const float *src = piv ? UT + kk * SU : DT + ci * SD;
                sfor<0, NT / 4>([&](auto Q) {
                    constexpr int j = c0 + PB + 4 * Q;
                    const float4 d = *(const float4 *)(src + 4 * Q);
                    z.M[0][j] = piv ? d.x : z.M[0][j] - d.x;
                    z.M[0][j + 1] = piv ? d.y : z.M[0][j + 1] - d.y;
                    z.M[0][j + 2] = piv ? d.z : z.M[0][j + 2] - d.z;
                    z.M[0][j + 3] = piv ? d.w : z.M[0][j + 3] - d.w;
                });
            }
            lds_fence();
        }
    });
    // pivot row k to lane k, as in lu_factor
    const int src = z.pivlane;
    sfor<0, NVP>([&](auto J) { z.M[0][J] = gather(z.M[0][J], src); });
    z.dinv[0] = gather(z.dinv[0], src);
    z.rs[0] = gather(z.rs[0], src);
}

template <int NVP, int L, class LT>
__device__ __forceinline__ void lu_factor(const Ctx &c, Zone<NVP, L, LT> &z)
{
    if constexpr (NVP == 48 && L == 64 && sizeof(LT) == 4) {
        if (c.lu_blocked) {
            lu_factor_blocked(c, z);
            return;
        }
    }
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    LT *prow = (LT *)(c.S + c.lay.prow);
    const int nv = own_copy(c.nv);
    sfor<0, RPL>([&](auto S) { z.pstep[S] = 127; });
    z.pivlane = c.gl;
    // The steps run in chunks of 8 (steps8); lanes past nvp hold zero rows and never pivot.
    auto step = [&](auto K) {
        constexpr int k = K;
        // the search runs in the factor's precision (FP32 values compare the same
        // way as their FP64 widenings, so the pivot is the same)
        LT bv = LT(-1);
        int bi = 1 << 20;
        sfor<0, RPL>([&](auto S) {
            int i = row_of<NVP, L>(c, S);
            LT a = fabs(z.M[S][k]);
            if (z.pstep[S] > k && i < NVP && a > bv) {
                bv = a;
                bi = i;
            }
        });
        LT gm = greduce<L>(bv, OpMax());
        int p;
        if constexpr (L == 64 && RPL == 1) {
            // one row per lane: the lowest flagged lane is the lowest row
            unsigned long long m = __ballot(bv == gm && bi < (1 << 20));
            p = m ? (int)__builtin_ctzll(m) : (1 << 20);
        } else if constexpr (RPL == 1 && L >= 2) {
            // the same within the group's L bits of the wave-wide mask
            const unsigned long long m = __ballot(bv == gm && bi < (1 << 20));
            const unsigned gm_bits =
                (unsigned)(m >> (threadIdx.x & (64 - L))) & (unsigned)((1ull << L) - 1ull);
            p = gm_bits ? (int)__builtin_ctz(gm_bits) : (1 << 20);
        } else {
            p = greduce<L>(bv == gm ? bi : (1 << 20), OpMin());
        }
        if constexpr (L == 64 && RPL == 1) {
            // Whole-wave zone: the pivot lane p is wave-uniform, so the pivot row is
            // read from its registers with v_readlane (8 columns at a time) instead of
            // going through LDS.
            const LT rinv = recip(lane_read(z.M[0][k], p));
            if (c.gl == p) {
                z.pstep[0] = k;
                z.dinv[0] = rinv;
            }
            const bool act = z.pstep[0] > k;
            const LT l = act ? z.M[0][k] * rinv : LT(0);
            if (act) z.M[0][k] = l;
            int pp = p;
            sfor<k + 1, NVP>([&](auto J) {
                if constexpr (J % 8 == 0) pp = after_s(pp, z.M[0][J - 1]);
                z.M[0][J] = fma(-l, lane_read(z.M[0][J], pp), z.M[0][J]);
            });
            if (c.gl == k) z.pivlane = p;
            return;
        }
        int pl = p & (L - 1);
        int ps = p / L;
        if constexpr (RPL == 1 && L >= 2) {
            // one row per lane: the pivot row is read from the pivot lane's registers through
            // the LDS crossbar (ds_bpermute), with no store and reload
            const int src = (int)(threadIdx.x & (64 - L)) + pl;
            LT pr[NVP];
            sfor<k, NVP>([&](auto J) { pr[J] = gather(z.M[0][J], src); });
            const LT rinv = recip(pr[k]);
            const int i = c.gl;
            if (i == p) {
                z.pstep[0] = k;
                z.dinv[0] = rinv;
            }
            const bool act = z.pstep[0] > k;
            const LT l = act ? z.M[0][k] * rinv : LT(0);
            if (act) z.M[0][k] = l;
            sfor<k + 1, NVP>([&](auto J) { z.M[0][J] = fma(-l, pr[J], z.M[0][J]); });
            if (c.gl == k) z.pivlane = p;
            return;
        }
        if (c.gl == pl) {
            sfor<k, NVP>([&](auto J) {
                if constexpr (RPL == 1) {
                    prow[J] = z.M[0][J];
                } else {
                    LT v = opq(z.M[0][J]);
                    sfor<1, RPL>([&](auto S) {
                        LT cand = opq(z.M[S][J]);
                        v = (ps == S) ? cand : v;
                    });
                    prow[J] = v;
                }
            });
        }
        lds_fence();
        LT rinv = recip(prow[k]);
        sfor<0, RPL>([&](auto S) {
            int i = row_of<NVP, L>(c, S);
            if (i == p) {
                z.pstep[S] = k;
                z.dinv[S] = rinv;
            }
            bool act = z.pstep[S] > k;
            LT l = act ? z.M[S][k] * rinv : LT(0);
            if (act) z.M[S][k] = l;
            sfor<k + 1, NVP>([&](auto J) {
                z.M[S][J] = fma(-l, prow[J], z.M[S][J]);
                // bound how many pivot-row loads are in flight (register pressure)
                if constexpr (NVP > 24 && J % 8 == 7) asm volatile("" ::: "memory");
            });
        });
        if constexpr (RPL == 1) {
            if (c.gl == k) z.pivlane = p;
        }
        lds_fence();
    };
    steps8<NVP>(nv, step);
    if constexpr (RPL == 1) {
        // Move pivot row k to group lane k: the factors become those of P M in natural
        // order, and the triangular solves broadcast from a fixed lane.
        const int src = (int)(threadIdx.x & (64 - L)) + z.pivlane;
        sfor<0, NVP>([&](auto J) { z.M[0][J] = gather(z.M[0][J], src); });
        z.dinv[0] = gather(z.dinv[0], src);
        if constexpr (sizeof(LT) == 4) z.rs[0] = gather(z.rs[0], src);
    }
}

// The LU in the pivot order of the zone's previous factorisation, one row a lane: lane k
// holds the k-th pivot row (form_M), so step k takes its pivot row from lane k by a
// broadcast within the group (DPP), with no search and no data-dependent exchange.  Each
// pivot must be at least PIV_KEEP times the largest candidate of its column (the rows not
// yet eliminated), the threshold test of threshold partial pivoting, checked lane by lane
// and reduced once at the end; a step that fails it makes the whole factorisation void
// (false), and the caller factors again with partial pivoting.  In exact arithmetic the
// solutions are the same for every pivot order.
constexpr float PIV_KEEP = 0.5f;

template <int NVP, int L, class LT>
__device__ __forceinline__ bool lu_kept_order(const Ctx &c, Zone<NVP, L, LT> &z)
{
    const int nv = own_copy(c.nv);
    bool bad = false;
    steps8<NVP>(nv, [&](auto K) {
        constexpr int k = K;
        const LT piv = bcast_k<L, k>(z.M[0][k]);
        // each candidate against the pivot in its own lane, so no reduction per step: the
        // rows of lanes below k are eliminated, lanes past nvp hold zero rows (a NaN fails)
        if (c.gl > k) bad = bad || !(fabs(z.M[0][k]) <= fabs(piv) * LT(1.0f / PIV_KEEP));
        const LT rinv = recip(piv);
        if (c.gl == k) z.dinv[0] = rinv;
        const bool act = c.gl > k;
        const LT l = act ? z.M[0][k] * rinv : LT(0);
        if (act) z.M[0][k] = l;
        sfor<k + 1, NVP>([&](auto J) { z.M[0][J] = fma(-l, bcast_k<L, k>(z.M[0][J]), z.M[0][J]); });
    });
    return !gany<L>(bad);
}

// M = I - gamma J and its LU factors: in the kept pivot order where the kernel keeps one,
// else (or when that order fails its threshold test) with partial pivoting from the natural
// order, whose pivot order is then kept.
template <int NVP, int L, class LT>
__device__ __forceinline__ void factor_M(const Ctx &c, Zone<NVP, L, LT> &z, double gamma)
{
    form_M(c, z, gamma);
    if constexpr (kept_order<NVP, L, LT>()) {
        if (!c.lu_blocked) {
            if (lu_kept_order(c, z)) return;
            z.pivlane = c.gl;
            form_M(c, z, gamma);
        }
    }
    lu_factor(c, z);
}

// Solve M x = b: b by local row in, x by local component out (same slots).
template <int NVP, int L, class LT>
__device__ __forceinline__ void lu_solve(const Ctx &c, const Zone<NVP, L, LT> &z, double (&b)[Zone<NVP, L, LT>::RPL])
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    constexpr bool MIXED = sizeof(LT) == 4;
    const int nv = own_copy(c.nv);
    if constexpr (RPL == 1) {
        // rows in pivot order (lu_factor): row k of L\U is in group lane k
        const int src = (int)(threadIdx.x & (64 - L)) + z.pivlane;
        const double bp = gather(b[0], src);
        LT v = MIXED ? (LT)(bp * (double)z.rs[0]) : (LT)bp;
        steps8<NVP>(nv, [&](auto K) {
            constexpr int k = K;
            const LT yk = bcast_k<L, k>(v);
            if (after(c.gl, v) > k) v = fma(-z.M[0][k], yk, v);
        });
        steps8<NVP, true>(nv, [&](auto K) {
            constexpr int k = K;
            const LT xk = bcast_k<L, k>(v * z.dinv[0]);
            if (after(c.gl, v) < k) v = fma(-z.M[0][k], xk, v);
        });
        double x = c.gl < nv ? (double)(v * z.dinv[0]) : 0.0;
        if (MIXED) x *= z.cs[0];
        b[0] = x;
        return;
    }
    LT bb[RPL], x[RPL];
    sfor<0, RPL>([&](auto S) {
        bb[S] = MIXED ? (LT)(b[S] * (double)z.rs[S]) : (LT)b[S];
        x[S] = LT(0);
    });
    steps8<NVP>(nv, [&](auto K) {
        constexpr int k = K;
        LT v = LT(0);
        bool own = false;
        int ps[RPL];
        sfor<0, RPL>([&](auto S) {
            ps[S] = after(z.pstep[S], bb[S]);
            LT cand = opq(bb[S]);
            if (ps[S] == k) { v = cand; own = true; }
        });
        LT zk = gbcast<L>(v, own);
        sfor<0, RPL>([&](auto S) {
            if (ps[S] > k) bb[S] = fma(-z.M[S][k], zk, bb[S]);
        });
    });
    steps8<NVP, true>(nv, [&](auto K) {
        constexpr int k = K;
        LT v = LT(0);
        bool own = false;
        int ps[RPL];
        sfor<0, RPL>([&](auto S) {
            ps[S] = after(z.pstep[S], bb[S]);
            LT cand = opq(bb[S]) * opq(z.dinv[S]);
            if (ps[S] == k) { v = cand; own = true; }
        });
        LT xk = gbcast<L>(v, own);
        sfor<0, RPL>([&](auto S) {
            if (ps[S] < k) bb[S] = fma(-z.M[S][k], xk, bb[S]);
        });
        if (c.gl == (k % L)) x[k / L] = xk;
    });
    sfor<0, RPL>([&](auto S) {
        double v = (double)x[S];
        if (MIXED) v *= z.cs[S];
        b[S] = v;
    });
}

// ------------------------------------------------------------ integrator

template <int NVP, int L, class LT>
__device__ __forceinline__ void rescale(Zone<NVP, L, LT> &z, double eta)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    // every order: the columns past q are zero (zeroed at the start, on an order decrease
    // and on a restart at order 1)
    double r = eta;
#pragma unroll
    for (int j = 1; j <= QMAX; ++j) {
#pragma unroll
        for (int s = 0; s < RPL; ++s) z.Z[j][s] *= r;
        r *= eta;
    }
}

// Error weights from the accepted state; also published to LDS for the FP32 scaling.
template <int NVP, int L, class LT>
__device__ __forceinline__ void set_weights(const Ctx &c, Zone<NVP, L, LT> &z)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    double *wb = c.S + c.lay.wbuf;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        int i = row_of<NVP, L>(c, s);
        double w = z.atol + z.rtol * fabs(z.Z[0][s]);
        z.iw[s] = (i < c.nv) ? zbm::recip_from(w, __builtin_amdgcn_rcp(w)) : 0.0;
        if (i < NVP) wb[i] = (i < c.nv) ? w : 1.0;
    }
}

// The history copy lives in LDS, one slot per (order, lane, local row), or per (order, row)
// in the trimmed layout; only this lane reads it back, so no exchange ordering is involved.
// Lanes past the last row hold no row (their history is identically zero) and no slot.
template <int NVP, int L, int RPL, class LT>
__device__ __forceinline__ bool zs_has(int gl)
{
    if constexpr (lds_trim(L, RPL, jac_f32(NVP, sizeof(LT) == 4)))
        return gl < NVP;
    else
        return true;
}

template <int NVP, int L, int RPL, class LT>
__device__ __forceinline__ int zs_slot(int gl, int j, int s)
{
    if constexpr (lds_trim(L, RPL, jac_f32(NVP, sizeof(LT) == 4)))
        return j * NVP + gl;
    else
        return (j * RPL + s) * L + gl;
}

template <int NVP, int L, class LT>
__device__ __forceinline__ void save_history(const Ctx &c, const Zone<NVP, L, LT> &z)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    double *zs = c.S + c.lay.zs;
#pragma unroll
    for (int j = 0; j <= QMAX; ++j)
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            if (zs_has<NVP, L, RPL, LT>(c.gl)) zs[zs_slot<NVP, L, RPL, LT>(c.gl, j, s)] = z.Z[j][s];
        }
}

template <int NVP, int L, class LT>
__device__ __forceinline__ void restore_history(const Ctx &c, Zone<NVP, L, LT> &z)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    const double *zs = c.S + c.lay.zs;
#pragma unroll
    for (int j = 0; j <= QMAX; ++j)
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            if (zs_has<NVP, L, RPL, LT>(c.gl)) z.Z[j][s] = zs[zs_slot<NVP, L, RPL, LT>(c.gl, j, s)];
        }
}

enum { RUNNING = -1 };

// Start of a zone: load, Hairer-Norsett-Wanner initial step.  Returns RUNNING or a status.
template <bool VC, int NVP, int L, class LT>
__device__ __forceinline__ int zone_start(const Ctx &c, Zone<NVP, L, LT> &z)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    const DevNet N = net_of(c);
    const Segment &SG = seg_of(c);
    const double *row = SG.state + c.zone * (N.ns + 1);
    const double *scale = SG.scale, *source = SG.source;
    double *ks = c.S + c.lay.ks;
    if (rates_in_lds<NVP, L, LT>(c)) {
        for (int r = c.gl; r < N.nr; r += L) {
            double s = scale ? scale[c.zone * N.nr + r] : 1.0;
            ks[r] = N.thermal ? s : s * exp(N.par[r].x);
        }
    }
    bool bad = false;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        int i = row_of<NVP, L>(c, s);
        double v = (i < N.nv) ? row[i] : 0.0;
        z.src[s] = (source && i < N.nv) ? source[c.zone * (N.ns + 1) + i] : 0.0;
        if (!isfinite(v) || !isfinite(z.src[s])) bad = true;
#pragma unroll
        for (int j = 0; j <= QMAX; ++j) z.Z[j][s] = 0.0;
        z.Z[0][s] = v;
        z.dyp[s] = 0.0;
    }
    z.nst = z.nje = z.nlu = z.nni = z.netf = z.ncf = 0;
    z.nfe = 0;
    z.have_j = z.have_m = 0;
    z.nst_j = z.nst_m = 0;
    z.pivlane = c.gl;   // the natural order: the first factorisation tests it
    z.gamma_m = 1.0;
    lds_fence();
    if (gany<L>(bad)) return ZB_ZONE_NONFINITE;
    set_weights(c, z);
    double f0[RPL], y1[RPL], f1[RPL];
    eval<false>(c, z, z.Z[0], f0);
    z.nfe = 1;
    bool badf = false;
#pragma unroll
    for (int s = 0; s < RPL; ++s)
        if (row_of<NVP, L>(c, s) < N.nv && !isfinite(f0[s])) badf = true;
    if (gany<L>(badf)) return ZB_ZONE_NONFINITE;
    double d0 = wrms(c, z, z.Z[0]);
    double d1 = wrms(c, z, f0);
    double ha = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
#pragma unroll
    for (int s = 0; s < RPL; ++s) y1[s] = z.Z[0][s] + ha * f0[s];
    eval<false>(c, z, y1, f1);
    z.nfe = 2;
#pragma unroll
    for (int s = 0; s < RPL; ++s) y1[s] = f1[s] - f0[s];
    double d2 = wrms(c, z, y1) / ha;
    double dm = fmax(d1, d2);
    double hb = (dm <= 1e-15) ? fmax(1e-6, ha * 1e-3) : sqrt(0.01 / dm);
    double h = fmin(fmin(100.0 * ha, hb), seg_of(c).dt);
    if (!isfinite(h) || !(h > 0.0)) return ZB_ZONE_NONFINITE;
    z.h = h;
    z.t = 0.0;
    z.q = 1;
    z.nequal = z.nefc = z.ncfc = 0;
#pragma unroll
    for (int s = 0; s < RPL; ++s) z.Z[1][s] = (c.jac_policy == METHOD_RKC) ? f0[s] : h * f0[s];
    if constexpr (VC) {
        if (c.gl == 0) c.S[c.lay.vc + VC_COUNT] = 0.0;   // no step history yet
        lds_fence();
    }
    return RUNNING;
}

// One step attempt.  Returns RUNNING, or the zone's final status.
// Newton iterations on the corrector with the current factors; z.f holds f at the
// prediction.  With factors formed at another gamma the correction is scaled by
// 2 / (1 + gamma / gamma_M).  Returns whether the iteration converged.
template <int NVP, int L, class LT>
__device__ __forceinline__ bool newton(const Ctx &c, Zone<NVP, L, LT> &z, double l0, double h, double tau)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    const double rc = h * l0 / z.gamma_m;
    const double cscale = (rc != 1.0) ? 2.0 / (1.0 + rc) : 1.0;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        z.y[s] = z.Z[0][s];
        z.dy[s] = 0.0;
    }
    double dprev = 0.0;
    for (int m = 0; m < 4; ++m) {
        if (m > 0) {
            eval<false>(c, z, z.y, z.f);
            z.nfe++;
        }
        double b[RPL];
#pragma unroll
        for (int s = 0; s < RPL; ++s) b[s] = -(z.dy[s] - l0 * (h * z.f[s] - z.Z[1][s]));
        lu_solve(c, z, b);
        if (cscale != 1.0) {
#pragma unroll
            for (int s = 0; s < RPL; ++s) b[s] *= cscale;
        }
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            z.y[s] += b[s];
            z.dy[s] += b[s];
        }
        double d = wrms(c, z, b);
        z.nni++;
        if (!isfinite(d)) return false;
        if (m == 0) {
            if (d <= tau) return true;
        } else {
            double rho = d / dprev;
            if (rho < 1.0 && rho * d / (1.0 - rho) <= tau) return true;
            // rho^(4-m) as products (m = 1, 2, 3): the same value as the power up to rounding
            const double rp = (m == 1) ? rho * rho * rho : ((m == 2) ? rho * rho : rho);
            if (rho >= 1.0 || rp * d / (1.0 - rho) > tau) return false;
        }
        dprev = d;
    }
    return false;
}

// Variable-coefficient form: xi_i = (t_{n+1} - t_{n+1-i}) / h from the accepted step sizes
// in LDS (unknown ones count as steps of the current h), l = coefficients of
// prod_{i<=q} (1 + x/xi_i) normalised to l_1 = 1, error divisor xi_{q+1}.  Returns l_0 and the
// divisor; the group's lane 0 leaves l_1..l_QMAX in LDS for the correction.
__device__ __forceinline__ void vc_coefficients(const Ctx &c, int q, double h, double &l0,
                                                double &ediv)
{
    double *vs = c.S + c.lay.vc;
    const int nh = (int)vs[VC_COUNT];
    const double rh = 1.0 / h;
    double xi[QMAX + 2];
    xi[1] = 1.0;
    double acc = 1.0;
#pragma unroll
    for (int i = 2; i <= QMAX + 1; ++i) {
        acc += (i - 2 < nh) ? vs[VC_HIST + i - 2] * rh : 1.0;
        xi[i] = acc;
    }
    double p[QMAX + 1];
    p[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= QMAX; ++j) p[j] = 0.0;
#pragma unroll
    for (int i = 1; i <= QMAX; ++i) {
        if (i <= q) {
            const double r = 1.0 / xi[i];
#pragma unroll
            for (int j = i; j >= 1; --j) p[j] = fma(p[j - 1], r, p[j]);
        }
    }
    const double r1 = 1.0 / p[1];
    l0 = r1;
    ediv = xi[2];
#pragma unroll
    for (int i = 3; i <= QMAX + 1; ++i) ediv = (i == q + 1) ? xi[i] : ediv;
    if (c.gl == 0) {
#pragma unroll
        for (int j = 1; j <= QMAX; ++j) vs[VC_L + j] = p[j] * r1;
    }
}

template <bool VC, bool HREGS, int NVP, int L, class LT>
__device__ __forceinline__ int zone_attempt(const Ctx &c, Zone<NVP, L, LT> &z)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    const double tau = 0.03;
    if (z.nst >= z.max_steps) return ZB_ZONE_MAXSTEPS;
    bool last = false;
    if (z.t + z.h >= seg_of(c).dt * (1.0 - 4.0 * DBL_EPSILON)) {
        double eta = (seg_of(c).dt - z.t) / z.h;
        rescale(z, eta);
        z.h = seg_of(c).dt - z.t;
        z.nequal = 0;
        last = true;
    }
    set_weights(c, z);
    // the history before the prediction: in registers of the attempt or in LDS (hist_regs)
    double Zs[HREGS ? QMAX + 1 : 1][RPL];
    if constexpr (HREGS) {
#pragma unroll
        for (int j = 0; j <= QMAX; ++j)
#pragma unroll
            for (int s = 0; s < RPL; ++s) Zs[j][s] = z.Z[j][s];
    } else {
        save_history(c, z);
    }
    auto restore = [&]() {
        if constexpr (HREGS) {
#pragma unroll
            for (int j = 0; j <= QMAX; ++j)
#pragma unroll
                for (int s = 0; s < RPL; ++s) z.Z[j][s] = Zs[j][s];
        } else {
            restore_history(c, z);
        }
    };
    // prediction: Pascal triangle, over every order (the columns past q are zero, so the
    // extra additions add zeros: no branch on q)
#pragma unroll
    for (int k = 0; k < QMAX; ++k)
#pragma unroll
        for (int j = QMAX; j > k; --j)
#pragma unroll
            for (int s = 0; s < RPL; ++s) z.Z[j - 1][s] += z.Z[j][s];

    const double h = z.h;
    double l0, ediv;
    if constexpr (VC) {
        vc_coefficients(c, z.q, h, l0, ediv);
    } else {
        l0 = inv_harmonic(z.q);
        ediv = (double)(z.q + 1);
    }
    const double gamma = h * l0;
    // f at the prediction, and the iteration matrix: formed on every attempt (policy 0),
    // or kept across steps and re-formed by the VODE rules (policy 1).  A second pass,
    // policy 1 only, refreshes a Jacobian from an earlier step after a Newton failure.
    // (Whole-wave zones take these branches uniformly; the compiler is told so.)
    bool conv = false, fresh = false;
    for (int pass = 0; pass < 2; ++pass) {
        bool new_j = true, new_m = true;
        if (c.jac_policy != 0 && pass == 0) {
            const double drc = z.have_m ? fabs(gamma / z.gamma_m - 1.0) : 1.0;
            new_m = group_uniform<L>(!z.have_m || drc > 0.3 || z.nst >= z.nst_m + 20);
            new_j = group_uniform<L>(new_m && (!z.have_j || z.nst >= z.nst_j + 50 || drc >= 0.2));
        }
        if (new_j) {
            if (group_uniform<L>(z.fdj != 0))
                fd_jacobian(c, z, z.Z[0], z.f);
            else
                eval<true>(c, z, z.Z[0], z.f);
            z.nje++;
            z.have_j = 1;
            z.nst_j = z.nst;
            fresh = true;
        } else {
            eval<false>(c, z, z.Z[0], z.f);
        }
        z.nfe++;
        if (new_m) {
            factor_M(c, z, gamma);
            z.nlu++;
            z.gamma_m = gamma;
            z.have_m = 1;
            z.nst_m = z.nst;
        }
        conv = newton(c, z, l0, h, tau);
        if (group_uniform<L>(conv || c.jac_policy == 0 || fresh)) break;
    }

    if (!conv) {
        restore();
        z.ncf++;
        if (++z.ncfc >= 10) return ZB_ZONE_CONV;
        rescale(z, 0.25);
        z.h *= 0.25;
        z.nequal = 0;
        if (z.t + z.h == z.t) return ZB_ZONE_HMIN;
        return RUNNING;
    }

    const double err = wrms(c, z, z.dy) / ediv;
    // Non-negativity of the abundances: a step that takes a species below -atol fails
    // like an error test and is cut to 0.9 of its feasible fraction (from the saved Z_0).
    double feas = 1.0;
    {
        const double *zs = c.S + c.lay.zs;
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            const int i = row_of<NVP, L>(c, s);
            if (i < c.ns && z.y[s] < -z.atol) {
                // Z_0 before the prediction
                const double old = HREGS ? Zs[0][s] : zs[zs_slot<NVP, L, RPL, LT>(c.gl, 0, s)];
                feas = fmin(feas, (old + z.atol) / (old - z.y[s]));
            }
        }
        feas = greduce<L>(feas, OpMin());
    }
    if (err > 1.0 || feas < 1.0) {
        restore();
        z.netf++;
        if (++z.nefc >= 10) return ZB_ZONE_ERRTEST;
        double eta = err > 1.0 ? fmax(0.1, step_factor(6.0 * err, z.q + 1)) : 1.0;
        if (feas < 1.0) eta = fmin(eta, fmax(0.1, 0.9 * feas));
        if (z.nefc >= 3) eta = 0.1;
        z.h *= eta;
        if (z.nefc >= 3) {
            z.q = 1;
            // the columns past the order stay zero (the prediction and the history copy run
            // over every order)
#pragma unroll
            for (int j = 2; j <= QMAX; ++j)
#pragma unroll
                for (int s = 0; s < RPL; ++s) z.Z[j][s] = 0.0;
            if constexpr (VC) {
                // the restarted history is a tangent, not past values
                if (c.gl == 0) c.S[c.lay.vc + VC_COUNT] = 0.0;
                lds_fence();
            }
            double f0[RPL];
            eval<false>(c, z, z.Z[0], f0);
            z.nfe++;
#pragma unroll
            for (int s = 0; s < RPL; ++s) z.Z[1][s] = z.h * f0[s];
        } else {
            rescale(z, eta);
        }
        z.nequal = 0;
        if (z.t + z.h == z.t) return ZB_ZONE_HMIN;
        return RUNNING;
    }

    // accept: Z_j += l_j e with e = dy / l_0, Z_0 = y
    const double H = VC ? 1.0 / l0 : harmonic(z.q);
#pragma unroll
    for (int j = 1; j <= QMAX; ++j) {
        const double lj = VC ? c.S[c.lay.vc + VC_L + j] : lcoef(z.q, j);
        const bool in = j <= z.q;
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            const double u = z.Z[j][s] + lj * (z.dy[s] * H);
            z.Z[j][s] = in ? u : z.Z[j][s];
        }
    }
    if constexpr (VC) {
        // the step just taken joins the history (newest first)
        lds_fence();
        if (c.gl == 0) {
            double *vs = c.S + c.lay.vc;
#pragma unroll
            for (int m = QMAX - 1; m > 0; --m) vs[VC_HIST + m] = vs[VC_HIST + m - 1];
            vs[VC_HIST] = h;
            vs[VC_COUNT] = fmin(vs[VC_COUNT] + 1.0, (double)QMAX);
        }
        lds_fence();
    }
#pragma unroll
    for (int s = 0; s < RPL; ++s) z.Z[0][s] = z.y[s];
    z.t = last ? seg_of(c).dt : z.t + h;
    z.nst++;
    z.nequal++;
    z.nefc = z.ncfc = 0;
    if (last) return ZB_ZONE_OK;

    if (z.nequal >= z.q + 1) {
        const int q = z.q;
        // eta_p = 1 / ((b E_p)^(1/(p+1)) + 1e-6) >= 1.5  iff  b E_p <= (2/3 - 1e-6)^(p+1).
        // The powers are evaluated only when some order may pass (a conservative
        // pre-filter, so every decision is the one the plain formula gives).
        const double cq = cpow23(q + 1) * (1.0 + 1e-9);
        bool may = 6.0 * err <= cq;
        double Em = 0.0, Ep = 0.0;
        if (q > 1) {
            double zq[RPL];
#pragma unroll
            for (int s = 0; s < RPL; ++s) {
                double v = 0.0;
#pragma unroll
                for (int j = 2; j <= QMAX; ++j) {
                    double cand = opq(z.Z[j][s]);
                    v = (j == q) ? cand : v;
                }
                zq[s] = v;
            }
            Em = factorial(q - 1) * wrms(c, z, zq);
            may = may || (6.0 * Em <= cpow23(q) * (1.0 + 1e-9));
        }
        if (q < QMAX) {
            double dd[RPL];
#pragma unroll
            for (int s = 0; s < RPL; ++s) dd[s] = z.dy[s] - z.dyp[s];
            Ep = wrms(c, z, dd) / (double)(q + 2);
            may = may || (10.0 * Ep <= cpow23(q + 2) * (1.0 + 1e-9));
        }
        double best = 0.0;
        int qnew = q;
        if (may) best = step_factor(6.0 * err, q + 1);
        if (may && q > 1) {
            double etam = step_factor(6.0 * Em, q);
            if (etam > best) { best = etam; qnew = q - 1; }
        }
        if (may && q < QMAX) {
            double etap = step_factor(10.0 * Ep, q + 2);
            if (etap > best) { best = etap; qnew = q + 1; }
        }
        if (best >= 1.5) {
            double eta = fmin(10.0, best);
            if (qnew == q + 1) {
                const double inv = 1.0 / factorial(q + 1);
#pragma unroll
                for (int s = 0; s < RPL; ++s) {
                    double zn = z.dy[s] * inv;
#pragma unroll
                    for (int j = 1; j <= QMAX; ++j) {
                        if (j <= q) z.Z[j][s] += stirling(q + 1, j) * zn;
                        if (j == q + 1) z.Z[j][s] = zn;
                    }
                }
                z.q = q + 1;
            } else if (qnew == q - 1) {
#pragma unroll
                for (int s = 0; s < RPL; ++s) {
                    double zq = 0.0;
#pragma unroll
                    for (int j = 2; j <= QMAX; ++j) {
                        double cand = opq(z.Z[j][s]);
                        zq = (j == q) ? cand : zq;
                    }
#pragma unroll
                    for (int j = 1; j < QMAX; ++j)
                        if (j < q) z.Z[j][s] -= stirling(q, j) * zq;
#pragma unroll
                    for (int j = 2; j <= QMAX; ++j)
                        if (j == q) z.Z[j][s] = 0.0;
                }
                z.q = q - 1;
            }
            rescale(z, eta);
            z.h *= eta;
            z.nequal = 0;
        }
    }
#pragma unroll
    for (int s = 0; s < RPL; ++s) z.dyp[s] = z.dy[s];
    return RUNNING;
}

// One step attempt of the damped second-order Runge-Kutta-Chebyshev method
// (Sommeijer, Shampine & Verwer; eps = 2/13), the integrator the paper names for
// mildly stiff zones.  Z_0 holds y_n and Z_1 holds F(y_n).  The number of stages
// comes from the Gershgorin bound of the Jacobian at y_n (assembled in LDS by the
// network code), the stage coefficients from the Chebyshev three-term recurrences
// (group-uniform scalars).  Error estimate (12 (y_n - y_{n+1}) + 6 h (F_n +
// F_{n+1})) / 15, step factor min(10, max(0.1, 0.8 err^(-1/3))), and the start, end
// clamp, abundance constraint and statuses of the BDF path.
template <int NVP, int L, class LT>
__device__ __forceinline__ int zone_attempt_rkc(const Ctx &c, Zone<NVP, L, LT> &z)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    constexpr int JS = NVP + 1;
    const DevNet N = net_of(c);
    if (z.nst >= z.max_steps) return ZB_ZONE_MAXSTEPS;
    bool last = false;
    double h = z.h;
    if (z.t + h >= seg_of(c).dt * (1.0 - 4.0 * DBL_EPSILON)) {
        h = seg_of(c).dt - z.t;
        last = true;
    }
    // spectral-radius bound: max over rows of sum_j |J_ij|
    {
        double tmp[RPL];
        eval<true>(c, z, z.Z[0], tmp);
        z.nje++;
    }
    lds_fence();
    const JacT<NVP, LT> *jb = (const JacT<NVP, LT> *)(c.S + c.lay.jbuf);
    double rs = 0.0;
    sfor<0, RPL>([&](auto S) {
        const int i = row_of<NVP, L>(c, S);
        if (i < N.nv) {
            double r = 0.0;
            for (int j = 0; j < N.nv; ++j) r += fabs((double)jb[i * JS + j]);
            rs = fmax(rs, r);
        }
    });
    const double rho = greduce<L>(rs, OpMax());
    const double hstab = ((double)(RKC_SMAX - 1) * (RKC_SMAX - 1) - 1.0) / (1.54 * rho);
    if (h > hstab) {
        h = hstab;
        last = false;
    }
    int ns = 1 + (int)floor(sqrt(1.0 + 1.54 * h * rho));
    ns = ns < 2 ? 2 : ns;
    // w1 = T_s'(w0) / T_s''(w0)
    const double w0 = 1.0 + (2.0 / 13.0) / ((double)ns * ns);
    double w1;
    {
        double t0 = 1.0, t1 = w0, d0 = 0.0, d1 = 1.0, e0 = 0.0, e1 = 0.0;
        for (int j = 2; j <= ns; ++j) {
            const double t2 = 2.0 * w0 * t1 - t0;
            const double d2 = 2.0 * t1 + 2.0 * w0 * d1 - d0;
            const double e2 = 4.0 * d1 + 2.0 * w0 * e1 - e0;
            t0 = t1; t1 = t2; d0 = d1; d1 = d2; e0 = e1; e1 = e2;
        }
        w1 = d1 / e1;
    }
    // stages; running T_j, T_j', T_j'' and b_j (b_0 = b_1 = b_2)
    double Y2[RPL], Y1[RPL], F[RPL];
    double T1 = w0, Tm = 1.0, D1 = 1.0, Dm = 0.0, E1 = 0.0, Em = 0.0;   // j-1 and j-2 values
    double T2 = 2.0 * w0 * T1 - Tm, D2 = 2.0 * T1 + 2.0 * w0 * D1 - Dm, E2 = 4.0 * D1 + 2.0 * w0 * E1 - Em;
    const double b2 = E2 / (D2 * D2);
    double bjm1 = b2, bjm2 = b2;   // b_1, b_0
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        Y2[s] = z.Z[0][s];
        Y1[s] = z.Z[0][s] + bjm1 * w1 * h * z.Z[1][s];
    }
    double Tjm1 = T1;              // T_{j-1}(w0) for j = 2
    double Tc = T1, Tp = Tm, Dc = D1, Dp = Dm, Ec = E1, Ep = Em;
    for (int j = 2; j <= ns; ++j) {
        const double Tn = 2.0 * w0 * Tc - Tp, Dn = 2.0 * Tc + 2.0 * w0 * Dc - Dp, En = 4.0 * Dc + 2.0 * w0 * Ec - Ep;
        const double bj = (j == 2) ? b2 : En / (Dn * Dn);
        const double mu = 2.0 * bj * w0 / bjm1;
        const double nu = -bj / bjm2;
        const double mut = 2.0 * bj * w1 / bjm1;
        const double gat = -(1.0 - bjm1 * Tjm1) * mut;
        eval<false>(c, z, Y1, F);
        z.nfe++;
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            const double yj = (1.0 - mu - nu) * z.Z[0][s] + mu * Y1[s] + nu * Y2[s] + mut * h * F[s] + gat * h * z.Z[1][s];
            Y2[s] = Y1[s];
            Y1[s] = yj;
        }
        Tp = Tc; Tc = Tn; Dp = Dc; Dc = Dn; Ep = Ec; Ec = En;
        Tjm1 = Tn;
        bjm2 = bjm1;
        bjm1 = bj;
    }
    // error estimate at y_{n+1} = Y1
    eval<false>(c, z, Y1, F);
    z.nfe++;
    double se = 0.0, feas = 1.0;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int i = row_of<NVP, L>(c, s);
        if (i < N.nv) {
            const double est = (12.0 * (z.Z[0][s] - Y1[s]) + 6.0 * h * (z.Z[1][s] + F[s])) / 15.0;
            const double w = z.atol + z.rtol * fmax(fabs(z.Z[0][s]), fabs(Y1[s]));
            const double x = est / w;
            se = fma(x, x, se);
            if (i < N.ns && Y1[s] < -z.atol)
                feas = fmin(feas, (z.Z[0][s] + z.atol) / (z.Z[0][s] - Y1[s]));
        }
    }
    double err = rms_of_sum(greduce<L>(se, OpAdd()), N.nv);
    feas = greduce<L>(feas, OpMin());
    if (!isfinite(err)) err = 1e10;
    // 0.8 err^(-1/3) (err finite and >= 0 here; err = 0 gives the cap)
    const double cr = kth_root(err, 3);
    double fac = fmin(10.0, fmax(0.1, cr > 0.0 ? 0.8 * zbm::recip_from(cr, __builtin_amdgcn_rcp(cr)) : 10.0));
    if (err > 1.0 || feas < 1.0) {
        z.netf++;
        if (++z.nefc >= 10) return ZB_ZONE_ERRTEST;
        if (feas < 1.0) fac = fmin(fac, fmax(0.1, 0.9 * feas));
        z.h = h * fmin(fac, 1.0);
        if (z.t + z.h == z.t) return ZB_ZONE_HMIN;
        return RUNNING;
    }
    z.nefc = 0;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        z.Z[0][s] = Y1[s];
        z.Z[1][s] = F[s];
    }
    z.t = last ? seg_of(c).dt : z.t + h;
    z.nst++;
    if (last) return ZB_ZONE_OK;
    z.h = h * fac;
    return RUNNING;
}

// The zone's counters, plus those of its first run while it is retried (in LDS) and, in the
// FP64 run of the fallback, those its mixed-precision run left in the stats row.
template <int NVP, int L, class LT>
__device__ __forceinline__ void write_stats(const Ctx &c, const Zone<NVP, L, LT> &z, bool add_row)
{
    int32_t *o = seg_of(c).stats + c.zone * 7;
    int add[7] = {0, 0, 0, 0, 0, 0, 0};
    if (z.tries > 0) {
        const int *cnt = (const int *)(c.S + c.lay.cnt);
        for (int k = 0; k < 7; ++k) add[k] = cnt[k];
    }
    if (add_row)
        for (int k = 0; k < 7; ++k) add[k] += o[k];
    o[0] = z.nst + add[0]; o[1] = z.nfe + add[1]; o[2] = z.nje + add[2]; o[3] = z.nlu + add[3];
    o[4] = z.nni + add[4]; o[5] = z.netf + add[5]; o[6] = z.ncf + add[6];
}

// Mixed-precision run with the FP64 fallback: a failed zone goes on its segment's list for
// the FP64 run, with its input row left as it is (results are written only when a zone ends)
// and its counters left in the stats row for that run to add.  False when the list is full;
// the zone then ends with its failure.
template <int NVP, int L, class LT>
__device__ __forceinline__ bool zone_defer(const Ctx &c, const Zone<NVP, L, LT> &z, int seg,
                                           const BurnArgs &A)
{
    const int lane = threadIdx.x & 63;
    unsigned long long idx = 0;
    if (c.gl == 0) idx = atomicAdd(A.fb + seg, 1ull);
    idx = (unsigned long long)__shfl((long long)idx, lane - c.gl, 64);
    if (idx >= (unsigned long long)FB_CAP) return false;
    if (c.gl == 0) {
        A.fb[MAXSEG + seg * FB_CAP + idx] = (unsigned long long)c.zone;
        if (seg_of(c).stats) write_stats(c, z, false);
    }
    return true;
}

template <int NVP, int L, class LT>
__device__ __forceinline__ void zone_finish(const Ctx &c, Zone<NVP, L, LT> &z, int status, const BurnArgs &A)
{
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    const int ns = c.ns;
    const bool replay = A.fb_mode == 2;
    if (replay && (status == ZB_ZONE_OK || status == ZB_ZONE_OK_RETRY)) status = ZB_ZONE_OK_FP64;
    if (status != ZB_ZONE_NONFINITE) {
        double *row = seg_of(c).state + c.zone * (ns + 1);
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            int i = row_of<NVP, L>(c, s);
            if (i < c.nv) row[i] = z.Z[0][s];
        }
    }
    if (c.gl == 0) {
        int32_t *st = seg_of(c).status;
        if (st) st[c.zone] = status;
        if (seg_of(c).stats) write_stats(c, z, replay);
        if (status != ZB_ZONE_OK && status != ZB_ZONE_OK_RETRY && status != ZB_ZONE_OK_FP64)
            atomicAdd(A.nfail, 1ull);
    }
}

template <class T>
__device__ __forceinline__ T uniform(T v)
{
    if constexpr (sizeof(T) == 8) {
        long long u;
        __builtin_memcpy(&u, &v, 8);
        int lo = __builtin_amdgcn_readfirstlane((int)(u & 0xffffffff));
        int hi = __builtin_amdgcn_readfirstlane((int)(u >> 32));
        u = (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
        __builtin_memcpy(&v, &u, 8);
        return v;
    } else {
        int u;
        __builtin_memcpy(&u, &v, 4);
        u = __builtin_amdgcn_readfirstlane(u);
        __builtin_memcpy(&v, &u, 4);
        return v;
    }
}

// Segment data for the wave (the wave works on one segment at a time, so it is uniform).
__device__ __forceinline__ void load_segment(Ctx &c, const BurnArgs &A, int seg, int nvp, int L,
                                             int rpl, bool vc, bool jf32, bool hregs)
{
    // seg is wave-uniform: scalar loads from the kernel-argument segment
    const BurnArgs *pa = (const BurnArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    const Segment &S = pa->seg[__builtin_amdgcn_readfirstlane(seg)];
    c.seg = __builtin_amdgcn_readfirstlane(seg);
    c.ns = uniform(S.net.ns);
    c.nv = uniform(S.net.nv);
    c.rates = pa->rates_lds != 0;
    c.lay = lds_layout(nvp, L, rpl, A.max_nr, vc, jf32, c.rates, hregs);
}

// Persistent kernel.  Each wave works through the segments in order; within a
// segment every group of L lanes pulls zones from the segment's queue until it
// is empty, and the wave moves on once all its groups have found it empty.
//
// Occupancy.  The 48-row kernels would take ~320 VGPRs and run one wave per
// SIMD; bounding them to two waves costs a few spilled registers and is ~20 %
// faster (the LU and solve chains are latency-bound).  The smaller kernels are
// left to the compiler (a bound there only adds spills).
template <int NVP, int L, int JP, class LT>
constexpr int min_waves_per_eu()
{
    // the reuse kernels keep the factors live across steps: bounded to two waves too
    // (but for the mixed 14-row ones below)
    // the 8-row kernel fits three waves with a Jacobian every step
    if (NVP == 8 && L == 8 && (JP == METHOD_BDF || JP == METHOD_BDF_VC)) return 3;
    // the mixed 14-row kernel with a Jacobian every step: three waves, at 168 VGPRs with
    // 156 bytes a lane spilled, ran 1.1 % faster than two (the FP64 one 15 % slower: more
    // spills; the same kernel without its list prefetch spilled less and ran 5 % slower).
    // The mixed reuse kernels too (268 bytes spilled), with the history copy in registers:
    // 11 % faster (fixed-coefficient form) and 2 % (variable-coefficient form)
    if (NVP == 14 && L == 16 && sizeof(LT) == 4 &&
        (JP == METHOD_BDF || JP == METHOD_BDF_REUSE || JP == METHOD_BDF_VC_REUSE))
        return 3;
    // the mixed 22-row kernel with a Jacobian every step (200 bytes spilled): 14 % faster
    if (NVP == 22 && L == 32 && sizeof(LT) == 4 && JP == METHOD_BDF) return 3;
    // RKC keeps no matrix: four waves fit (the compiler would take two registers more)
    if (JP == METHOD_RKC) return 4;
    return ((NVP >= 48 && L == 64) || (method_jac(JP) == 1 && L >= 16)) ? 2 : 1;
}

template <int NVP, int L, class LT, int JP>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(min_waves_per_eu<NVP, L, JP, LT>())))
void burn_kernel(BurnArgs A)
{
    extern __shared__ double smem[];
    constexpr int RPL = Zone<NVP, L, LT>::RPL;
    const int lane = threadIdx.x & 63;
    Ctx c;
    c.gl = lane & (L - 1);
    const int g = lane / L;
    Zone<NVP, L, LT> z;
    int seg = 0;
    c.jac_policy = JP == METHOD_RKC ? METHOD_RKC : method_jac(JP);
    c.lu_blocked = method_blocked_lu(JP);   // a constant: each
                         // method is its own kernel (the reuse keeps the
                         // factors live across steps, which costs registers)
    load_segment(c, A, seg, NVP, L, RPL, method_vc(JP), jac_f32(NVP, sizeof(LT) == 4),
                 hist_regs(NVP, L, sizeof(LT) == 4, JP));
    c.S = smem + g * c.lay.total;
    // zones of a segment: its own, or in the FP64 run of the fallback those on its list
    auto seg_zones = [&](int sg) -> int64_t {
        const BurnArgs *pa = (const BurnArgs *)__builtin_amdgcn_kernarg_segment_ptr();
        if (A.fb_mode == 2) {
            const unsigned long long n = pa->fb[sg];
            return (int64_t)(n < (unsigned long long)FB_CAP ? n : (unsigned long long)FB_CAP);
        }
        return pa->seg[sg].zones;
    };
    int64_t zones = uniform(seg_zones(0));
    bool need = true, dry = false;
    for (;;) {
        if (need && !dry) {
            unsigned long long item = 0;
            if (c.gl == 0) item = atomicAdd(A.queue + seg, 1ull);
            item = (unsigned long long)__shfl((long long)item, lane - c.gl, 64);
            if (item >= (unsigned long long)zones) {
                dry = true;
            } else {
                c.zone = A.fb_mode == 2 ? (int64_t)A.fb[MAXSEG + seg * FB_CAP + item] : (int64_t)item;
                z.rtol = seg_of(c).rtol;
                z.atol = seg_of(c).atol;
                z.max_steps = A.max_steps;
                z.tries = 0;
                z.fdj = 0;
                int st = zone_start<method_vc(JP)>(c, z);
                if (st == RUNNING)
                    need = false;
                else
                    zone_finish(c, z, st, A);
            }
        }
        if (__ballot(!dry) == 0) {
            if (++seg >= A.nseg) break;
            load_segment(c, A, seg, NVP, L, RPL, method_vc(JP), jac_f32(NVP, sizeof(LT) == 4),
                 hist_regs(NVP, L, sizeof(LT) == 4, JP));
            c.S = smem + g * c.lay.total;
            zones = uniform(seg_zones(__builtin_amdgcn_readfirstlane(seg)));
            need = true;
            dry = false;
            continue;
        }
        if (!need) {
            int st = (JP == METHOD_RKC) ? zone_attempt_rkc(c, z)
                                        : zone_attempt<method_vc(JP), hist_regs(NVP, L, sizeof(LT) == 4, JP)>(c, z);
            if (st != RUNNING) {
                if (st != ZB_ZONE_OK && A.retry && z.tries == 0) {
                    // Zone-by-zone retry with the retry tolerances, from the zone's input
                    // (still in memory: results are written only when a zone ends).  The
                    // first run's counters wait in LDS and are added at the end.
                    if (c.gl == 0) {
                        int *cnt = (int *)(c.S + c.lay.cnt);
                        cnt[0] = z.nst; cnt[1] = z.nfe; cnt[2] = z.nje; cnt[3] = z.nlu;
                        cnt[4] = z.nni; cnt[5] = z.netf; cnt[6] = z.ncf;
                    }
                    z.rtol = A.retry_rtol;
                    z.atol = A.retry_atol;
                    z.max_steps = A.retry_max_steps;
                    z.tries = 1;
                    z.fdj = A.retry_jac;
                    st = zone_start<method_vc(JP)>(c, z);
                    if (st == RUNNING) continue;
                } else if (st == ZB_ZONE_OK && z.tries > 0) {
                    st = ZB_ZONE_OK_RETRY;
                }
                if (A.fb_mode == 1 && st != ZB_ZONE_OK && st != ZB_ZONE_OK_RETRY &&
                    zone_defer(c, z, seg, A)) {
                    need = true;
                    continue;
                }
                zone_finish(c, z, st, A);
                need = true;
            }
        }
    }
}

#define ZB_K(NVP, L, LT, MIX) {NVP, L, MIX, 0, (const void *)&burn_kernel<NVP, L, LT, 0>}
#define ZB_KR(NVP, L, LT, MIX) {NVP, L, MIX, 1, (const void *)&burn_kernel<NVP, L, LT, 1>}
#define ZB_KC(NVP, L) {NVP, L, 0, 2, (const void *)&burn_kernel<NVP, L, double, 2>}
#define ZB_KV(NVP, L, LT, MIX) {NVP, L, MIX, 3, (const void *)&burn_kernel<NVP, L, LT, 3>}
#define ZB_KVR(NVP, L, LT, MIX) {NVP, L, MIX, 4, (const void *)&burn_kernel<NVP, L, LT, 4>}
#define ZB_KB(NVP, L) {NVP, L, 1, 5, (const void *)&burn_kernel<NVP, L, float, 5>}
#define ZB_KVB(NVP, L) {NVP, L, 1, 6, (const void *)&burn_kernel<NVP, L, float, 6>}

}  // namespace zb

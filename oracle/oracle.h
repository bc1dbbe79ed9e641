/*
 * CPU FP64 oracle for the per-zone stiff BDF burn.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library.  It shares no
 * code, header, table or constant with the HIP path under
 * paper_2608_06466_amd/, and it is deliberately plain: scalar loops, FP64,
 * built with contraction off, no SIMD, no blocking.
 *
 * What it computes (the paper, "Software design": one zone at a time, zones
 * independent, a VODE-type stiff integrator, failures returned to the caller
 * after a step cap):
 *   each zone integrates y' = f(y) over [0, dt] with a variable-order (1..5)
 *   BDF method in Nordsieck form, Newton iteration on a dense LU of
 *   M = I - gamma J with the analytic Jacobian, and weighted-RMS error,
 *   order and step control.  The exact rules are in bdf.c.
 */
#ifndef ZB_ORACLE_H
#define ZB_ORACLE_H

#include <complex.h>
#include <stdint.h>

#define ORC_NVMAX 64
#define ORC_QMAX 5

enum { ORC_OK = 0, ORC_MAXSTEPS = 1, ORC_ERRTEST = 2, ORC_CONV = 3, ORC_HMIN = 4, ORC_NONFINITE = 5,
       ORC_OK_RETRY = 6 /* failed, then succeeded on the retry */ };

typedef struct {
    int ns;            /* species */
    int thermal;       /* 1: T (state slot ns) is integrated and drives the rates */
    int nr;            /* reactions */
    const int32_t *reactant;  /* [nr][2], second -1 for first order */
    const int32_t *product;   /* [nr][2], second -1 for a single product */
    const double *lnA, *n_exp, *E, *q;   /* [nr] */
} orc_net;

typedef struct { int32_t nst, nfe, nje, nlu, nni, netf, ncf; } orc_stats;

int orc_nvar(const orc_net *net);
int orc_check_net(const orc_net *net);

/* Network: rate constants, right-hand side, analytic Jacobian (row-major nv x nv). */
void orc_rates(const orc_net *net, const double *scale, const double *y, double *k, double *dkdT);
void orc_rhs(const orc_net *net, const double *scale, const double *y, double *f);
void orc_rhs_cplx(const orc_net *net, const double *scale, const double complex *y, double complex *f);
void orc_jac(const orc_net *net, const double *scale, const double *y, double *J);

/* Dense LU with partial pivoting, ties to the lowest row.  Returns 0, or k+1 for a zero pivot at step k. */
int orc_lu(int n, double *A, int *piv);
void orc_lu_solve(int n, const double *LU, const int *piv, double *b);

/* BDF coefficients and Nordsieck order changes. */
void orc_lcoef(int q, double *l);
void orc_stirling(int n, double *c);
void orc_order_raise(int nv, int q, double *Z, const double *dy);
void orc_order_lower(int nv, int q, double *Z);

/* Burn one zone in place (row = [ns species, T]).  Returns the zone status. */
int orc_burn_zone(const orc_net *net, double *row, const double *scale, double dt,
                  double rtol, double atol, int max_steps, orc_stats *st);
/* Burn zones [zones][ns+1] in place; scale is [zones][nr] or NULL; stats [zones][7] or NULL. */
int orc_burn(const orc_net *net, double *state, int64_t zones, const double *scale, double dt,
             double rtol, double atol, int max_steps, int32_t *status, int32_t *stats, int nthreads);

/* The same with a constant source per zone added to the right-hand side (the simplified
   spectral-deferred-correction coupling the paper names: the hydro's advective change per
   unit time enters the burn as a fixed term).  source is [zones][ns+1] (the T entry is used
   only by thermal networks) or NULL. */
int orc_burn_zone_src(const orc_net *net, double *row, const double *scale, const double *src,
                      double dt, double rtol, double atol, int max_steps, orc_stats *st);
int orc_burn_src(const orc_net *net, double *state, int64_t zones, const double *scale,
                 const double *source, double dt, double rtol, double atol, int max_steps,
                 int32_t *status, int32_t *stats, int nthreads);

/* Fixed step, fixed order: nsteps BDF-q steps of size h from the Nordsieck array Z[q+1][nv];
   ys[n] = y after step n, errs[n] = its local error estimate (weights atol 1e-12, rtol 1e-8). */
int orc_fixed_steps(const orc_net *net, const double *scale, int q, double h, int nsteps,
                    double *Z, double *ys, double *errs);

/* Brute force: 2-stage Radau IIA on a geometric mesh (first step h0), full Newton. */
int orc_radau(const orc_net *net, const double *scale, double *y, double dt, int64_t nsteps, double h0);

/* Runge-Kutta-Chebyshev integrator (rkc.c): the damped second-order method for mildly stiff
   zones, with the same state layout, statuses and counters as the BDF burn. */
#define ORC_RKC_SMAX 250
int orc_rkc_stages(double h, double rho);
int orc_rkc_fixed(const orc_net *net, const double *scale, double *y, double h, int nsteps, int s);
int orc_rkc_zone(const orc_net *net, double *row, const double *scale, const double *src, double dt,
                 double rtol, double atol, int max_steps, orc_stats *st);
int orc_rkc(const orc_net *net, double *state, int64_t zones, const double *scale, const double *source,
            double dt, double rtol, double atol, int max_steps, int32_t *status, int32_t *stats,
            int nthreads);

/* Zone-by-zone retry of failed zones (the paper: retry an integration with different
   tolerances).  enabled = 0 turns it off. */
/* jac: the retry's Jacobian, 0 analytic (as in the first run), 1 finite differences
   (orc_fd_jac). */
typedef struct { int enabled; double rtol, atol; int max_steps; int jac; } orc_retry;
int orc_burn_retry(const orc_net *net, double *state, int64_t zones, const double *scale,
                   const double *source, double dt, double rtol, double atol, int max_steps,
                   const orc_retry *retry, int32_t *status, int32_t *stats, int nthreads);

/* jac_policy 0: Jacobian and LU on every step attempt (the default everywhere above).
   jac_policy 1: VODE-style reuse of the iteration matrix and the Jacobian (rules in bdf.c). */
/* vc: 0 the fixed-leading-coefficient form (the default everywhere above), 1 the
   variable-coefficient form (l and the error divisor from the step history, bdf.c). */
int orc_burn_zone_ex(const orc_net *net, double *row, const double *scale, const double *src,
                     double dt, double rtol, double atol, int max_steps, int jac_policy,
                     int fd_jac, int vc, orc_stats *st);
void orc_vc_xi(int q, double h, const double *hist, int nh, double *xi);
void orc_vc_lcoef(int q, const double *xi, double *l);
int orc_vc_steps(const orc_net *net, const double *scale, int q, int nsteps, const double *hs,
                 const double *hist0, int nh0, double *Zio, double *ys);
/* Finite-difference Jacobian of f (the network RHS plus src, if any) at y, row-major
   [nv][nv]: column j is (f(y + d_j e_j) - f(y)) / d_j with d_j = 2^-26 max(|y_j|,
   atol + rtol |y_j|), taken as (y_j + d_j) - y_j. */
void orc_fd_jac(const orc_net *net, const double *scale, const double *src, const double *y,
                double rtol, double atol, double *J);
int orc_burn_ex(const orc_net *net, double *state, int64_t zones, const double *scale,
                const double *source, double dt, double rtol, double atol, int max_steps,
                int jac_policy, int form, const orc_retry *retry, int32_t *status,
                int32_t *stats, int nthreads);

#endif

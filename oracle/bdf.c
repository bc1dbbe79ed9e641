/*
 * Oracle BDF integrator (test infrastructure only; see oracle.h).
 *
 * The paper names VODE (Brown, Byrne & Hindmarsh 1989) as its stiff
 * integrator and states none of its rules.  This file is the reading used by
 * the whole project, written from the published theory of Nordsieck-form BDF
 * methods (fixed leading coefficient, interpolatory rescaling):
 *
 *  Norm     |v| = sqrt(mean_i (v_i / w_i)^2), w_i = atol + rtol |y_i| taken from
 *           the last accepted y and held for the whole step attempt.
 *  History  Z_j = h^j y^(j) / j!, j = 0..q (q <= 5).  Prediction multiplies Z
 *           by the Pascal matrix.  l(q) = coefficients of prod_{i<=q}(1 + x/i),
 *           divided by the harmonic number H_q so that l_1 = 1; gamma = h l_0.
 *  Start    The Hairer-Norsett-Wanner initial step estimate with order 1.
 *  Newton   At most 4 iterations on  dy - l_0 (h f(y0 + dy) - Z_1) = 0  with
 *           M = I - gamma J and J taken at the prediction.  With d_m the norm of
 *           the m-th correction and rho = d_m / d_{m-1}: converged when d_0 <= tau
 *           or, later, rho < 1 and rho d_m / (1 - rho) <= tau; failed when rho >= 1
 *           or rho^(4-m) d_m / (1 - rho) > tau (no convergence within 4), or on a
 *           non-finite norm or a zero pivot.  tau = 0.03 (Hairer-Wanner kappa).
 *  Error    E_q = |dy| / (q+1); a step is accepted when E_q <= 1.
 *  Control  (order and step selection after the Nordsieck/LSODE family, with
 *           biased estimates) After q+1 accepted steps at the same h and q, and
 *           after every further step while nothing changes, form
 *             E_{q-1} = (q-1)! |Z_q|,  E_q,  E_{q+1} = |dy - dy_prev| / (q+2),
 *             eta_p = 1 / ((b_p E_p)^(1/(p+1)) + 1e-6),  b = 6, 6, 10;
 *           take the largest (ties keep q, then prefer q-1); change nothing when
 *           it is below 1.5, else eta = min(10, eta_p).  Order changes keep Z the
 *           interpolant of the last accepted values (Stirling coefficients).
 *  Failure  Newton failure: restore Z, h *= 0.25.  Error-test failure: restore Z,
 *           eta = max(0.1, 1 / ((6 E_q)^(1/(q+1)) + 1e-6)); from the third
 *           consecutive one, eta = 0.1 and the history restarts at order 1 from
 *           f at the accepted state.  Ten consecutive failures of either kind end
 *           the zone (CONV or ERRTEST); t + h == t ends it (HMIN); max_steps
 *           accepted steps end it (MAXSTEPS); a non-finite start ends it
 *           (NONFINITE).  A failed zone keeps its last accepted state.
 *  End      The step that would reach dt (within 4 eps relative) is shortened
 *           to land on dt exactly.
 *  Form     (option) The variable-coefficient form takes l and the error divisor
 *           from the step history instead (coef_variable).  Order changes keep the
 *           fixed coefficients: they happen only after q+1 steps of equal size, where
 *           the two forms coincide.
 */
#include <float.h>
#include <math.h>
#include <string.h>

#include "oracle.h"

typedef struct {
    const orc_net *net;
    const double *scale;
    int nv;
    const double *src;   /* constant source added to f (nv entries), or NULL */
} sys_t;

static double wrms(int nv, const double *v, const double *w)
{
    double s = 0.0;
    for (int i = 0; i < nv; i++) {
        double x = v[i] / w[i];
        s += x * x;
    }
    return sqrt(s / nv);
}

/* Coefficients of one step attempt: l(q) (l_1 = 1, gamma = h l_0) and the divisor of the
   local-error estimate.  The fixed-leading-coefficient form takes l from prod (1 + x/i) and
   divides by q + 1; the variable-coefficient form (below) from the step history. */
typedef struct {
    double l[ORC_QMAX + 1];
    double ediv;
} coef_t;

/* Estimated local error of the accepted BDF-q step: |dy| / (q+1), or / xi_{q+1}. */
static double local_error(int nv, const coef_t *C, const double *dy, const double *w)
{
    return wrms(nv, dy, w) / C->ediv;
}

/* f(y) = network RHS + the zone's constant source (the simplified-SDC coupling of a
   hydro update: the advective change per unit time held fixed over the burn). */
static void rhs(const sys_t *S, const double *y, double *f, orc_stats *st)
{
    orc_rhs(S->net, S->scale, y, f);
    if (S->src)
        for (int i = 0; i < S->nv; i++) f[i] += S->src[i];
    st->nfe++;
}

/* l(q): prod_{i=1..q} (1 + x/i), normalised by its x coefficient (= H_q). */
void orc_lcoef(int q, double *l)
{
    double p[ORC_QMAX + 2] = {1.0};
    for (int i = 1; i <= q; i++) {
        for (int j = i; j >= 1; j--) p[j] += p[j - 1] / i;
    }
    for (int j = 0; j <= q; j++) l[j] = p[j] / p[1];
}

/* c(n, j) = [x^j] x (x+1) ... (x+n-1)  (unsigned Stirling numbers of the first kind). */
void orc_stirling(int n, double *c)
{
    double p[ORC_QMAX + 3] = {0.0};
    p[1] = 1.0;                      /* the factor x */
    for (int m = 1; m < n; m++) {    /* multiply by (x + m) */
        for (int j = m + 1; j >= 1; j--) p[j] = p[j - 1] + m * p[j];
        p[0] = m * p[0];
    }
    for (int j = 0; j <= n; j++) c[j] = p[j];
}

static void coef_fixed(int q, coef_t *C)
{
    orc_lcoef(q, C->l);
    C->ediv = q + 1;
}

/* Variable-coefficient BDF (the form of VODE): with xi_i = (t_{n+1} - t_{n+1-i}) / h the
   corrector direction is prod_{i<=q} (1 + x/xi_i), the polynomial that vanishes at the q
   past points, so the corrected Nordsieck polynomial keeps interpolating the last q+1
   values and the step is the BDF on the actual (uneven) grid; normalised to l_1 = 1.  The
   error estimate divides by xi_{q+1} (q + 1 at constant steps).  hist[m] = t_{n-m} -
   t_{n-m-1} for the nh known past steps; unknown ones count as steps of the current h, so
   the start and a restart use the fixed coefficients. */
void orc_vc_xi(int q, double h, const double *hist, int nh, double *xi)
{
    double acc = 1.0;
    xi[1] = 1.0;
    for (int i = 2; i <= q + 1; i++) {
        acc += (i - 2 < nh) ? hist[i - 2] / h : 1.0;
        xi[i] = acc;
    }
}

void orc_vc_lcoef(int q, const double *xi, double *l)
{
    double p[ORC_QMAX + 2] = {1.0};
    for (int i = 1; i <= q; i++)
        for (int j = i; j >= 1; j--) p[j] += p[j - 1] / xi[i];
    for (int j = 0; j <= q; j++) l[j] = p[j] / p[1];
}

static void coef_variable(int q, double h, const double *hist, int nh, coef_t *C)
{
    double xi[ORC_QMAX + 2];
    orc_vc_xi(q, h, hist, nh, xi);
    orc_vc_lcoef(q, xi, C->l);
    C->ediv = xi[q + 1];
}

/* Raise q -> q+1: the new leading term is dy / (q+1)!, added along x(x+1)...(x+q). */
void orc_order_raise(int nv, int q, double *Z, const double *dy)
{
    double c[ORC_QMAX + 3];
    double fact = 1.0;
    for (int i = 2; i <= q + 1; i++) fact *= i;
    orc_stirling(q + 1, c);
    double *Zn = Z + (size_t)(q + 1) * nv;
    for (int i = 0; i < nv; i++) Zn[i] = dy[i] / fact;
    for (int j = 1; j <= q; j++)
        for (int i = 0; i < nv; i++) Z[(size_t)j * nv + i] += c[j] * Zn[i];
}

/* Lower q -> q-1: remove the leading term along x(x+1)...(x+q-1). */
void orc_order_lower(int nv, int q, double *Z)
{
    double c[ORC_QMAX + 3];
    orc_stirling(q, c);
    const double *Zq = Z + (size_t)q * nv;
    for (int j = 1; j < q; j++)
        for (int i = 0; i < nv; i++) Z[(size_t)j * nv + i] -= c[j] * Zq[i];
    for (int i = 0; i < nv; i++) Z[(size_t)q * nv + i] = 0.0;
}

static void rescale(int nv, int q, double *Z, double eta)
{
    double r = eta;
    for (int j = 1; j <= q; j++) {
        for (int i = 0; i < nv; i++) Z[(size_t)j * nv + i] *= r;
        r *= eta;
    }
}

static void predict(int nv, int q, double *Z)
{
    for (int k = 0; k < q; k++)
        for (int j = q; j > k; j--)
            for (int i = 0; i < nv; i++) Z[(size_t)(j - 1) * nv + i] += Z[(size_t)j * nv + i];
}

/* Iteration-matrix state of a zone.  Policy 0 (the default) evaluates J and factors
   M = I - gamma J on every step attempt.  Policy 1 is the VODE-style reuse of the
   Brown-Byrne-Hindmarsh paper: M is kept across steps and re-formed only when gamma has
   changed by more than 30 % since it was formed, after 20 steps, or after a Newton
   failure with a Jacobian from an earlier step; a re-formed M evaluates a fresh J unless
   the saved one is younger than 50 steps and gamma moved by less than 20 % (an age-only
   refresh).  With M formed at gamma_M != gamma the Newton correction is scaled by
   2 / (1 + gamma / gamma_M), the factor VODE applies to a lagged matrix. */
typedef struct {
    int policy;
    int fd;                      /* 1: finite-difference Jacobian (a retry's alternative) */
    double rtol, atol;           /* the run's tolerances (they scale the differences) */
    int have_j, have_m;
    int nst_j, nst_m;            /* nst when J was evaluated / M was factored */
    double gamma_m;
    int sing;
    double J[ORC_NVMAX * ORC_NVMAX], LU[ORC_NVMAX * ORC_NVMAX];
    int piv[ORC_NVMAX];
} jac_t;

static void form_lu(const sys_t *S, jac_t *J, double gamma, orc_stats *st)
{
    int nv = S->nv;
    for (int i = 0; i < nv; i++)
        for (int j = 0; j < nv; j++) J->LU[i * nv + j] = (i == j ? 1.0 : 0.0) - gamma * J->J[i * nv + j];
    J->sing = orc_lu(nv, J->LU, J->piv);
    st->nlu++;
    J->gamma_m = gamma;
    J->have_m = 1;
    J->nst_m = st->nst;
}

/* Finite-difference Jacobian: the other Jacobian approximation the paper names for a
   zone-by-zone retry (Software design).  Forward differences in each variable with the
   step d_j = 2^-26 max(|y_j|, atol + rtol |y_j|) (the square root of the FP64 unit
   roundoff times the variable's scale), replaced by (y_j + d_j) - y_j so that it is
   exactly the change applied.  The nv perturbed evaluations count as RHS evaluations;
   f(y) itself is the RHS at the prediction, which Newton counts. */
static void fd_jac(const sys_t *S, const double *y, double rtol, double atol, double *Jm,
                   orc_stats *st)
{
    int nv = S->nv;
    double f0[ORC_NVMAX], f1[ORC_NVMAX], yp[ORC_NVMAX];
    orc_stats uncounted;
    rhs(S, y, f0, &uncounted);
    for (int j = 0; j < nv; j++) {
        for (int i = 0; i < nv; i++) yp[i] = y[i];
        double d = ldexp(1.0, -26) * fmax(fabs(y[j]), atol + rtol * fabs(y[j]));
        yp[j] = y[j] + d;
        d = yp[j] - y[j];
        rhs(S, yp, f1, st);
        for (int i = 0; i < nv; i++) Jm[i * nv + j] = (f1[i] - f0[i]) / d;
    }
}

void orc_fd_jac(const orc_net *net, const double *scale, const double *src, const double *y,
                double rtol, double atol, double *J)
{
    sys_t S = {net, scale, orc_nvar(net), src};
    orc_stats st;
    fd_jac(&S, y, rtol, atol, J, &st);
}

static void eval_jac(const sys_t *S, jac_t *J, const double *y, orc_stats *st)
{
    if (J->fd)
        fd_jac(S, y, J->rtol, J->atol, J->J, st);
    else
        orc_jac(S->net, S->scale, y, J->J);
    st->nje++;
    J->have_j = 1;
    J->nst_j = st->nst;
}

/* The Newton iterations with the current M.  Returns 0 on convergence, 1 on failure. */
static int newton_iter(const sys_t *S, const jac_t *J, const coef_t *C, double h, const double *Z,
                       const double *w, double *y, double *dy, orc_stats *st)
{
    int nv = S->nv;
    double f[ORC_NVMAX], b[ORC_NVMAX];
    const double *l = C->l;
    const double gamma = h * l[0];
    const double rc = gamma / J->gamma_m;          /* 1 with a matrix formed at this gamma */
    const double cscale = (rc != 1.0) ? 2.0 / (1.0 + rc) : 1.0;
    const double tau = 0.03;
    for (int i = 0; i < nv; i++) { y[i] = Z[i]; dy[i] = 0.0; }
    double dprev = 0.0;
    for (int m = 0; m < 4; m++) {
        rhs(S, y, f, st);
        for (int i = 0; i < nv; i++) b[i] = -(dy[i] - l[0] * (h * f[i] - Z[nv + i]));
        if (J->sing) return 1;
        orc_lu_solve(nv, J->LU, J->piv, b);
        if (cscale != 1.0)
            for (int i = 0; i < nv; i++) b[i] *= cscale;
        for (int i = 0; i < nv; i++) { y[i] += b[i]; dy[i] += b[i]; }
        double d = wrms(nv, b, w);
        st->nni++;
        if (!isfinite(d)) return 1;
        if (m == 0) {
            if (d <= tau) return 0;
        } else {
            double rho = d / dprev;
            if (rho < 1.0 && rho * d / (1.0 - rho) <= tau) return 0;
            if (rho >= 1.0 || pow(rho, 4 - m) * d / (1.0 - rho) > tau) return 1;
        }
        dprev = d;
    }
    return 1;
}

/* One Newton solve of the corrector.  On success dy holds y - y_pred and y the new value.
   Returns 0 on convergence, 1 on failure. */
static int newton(const sys_t *S, jac_t *J, const coef_t *C, double h, const double *Z,
                  const double *w, double *y, double *dy, orc_stats *st)
{
    const double gamma = h * C->l[0];
    if (J->policy == 0) {
        eval_jac(S, J, Z, st);
        form_lu(S, J, gamma, st);
        return newton_iter(S, J, C, h, Z, w, y, dy, st);
    }
    int fresh = 0;   /* J evaluated at this attempt's prediction */
    const double drc = J->have_m ? fabs(gamma / J->gamma_m - 1.0) : 1.0;
    if (!J->have_m || drc > 0.3 || st->nst >= J->nst_m + 20) {
        if (!J->have_j || st->nst >= J->nst_j + 50 || drc >= 0.2) {
            eval_jac(S, J, Z, st);
            fresh = 1;
        }
        form_lu(S, J, gamma, st);
    }
    if (newton_iter(S, J, C, h, Z, w, y, dy, st) == 0) return 0;
    if (fresh) return 1;
    /* failure with a Jacobian from an earlier step: refresh it here and retry once */
    eval_jac(S, J, Z, st);
    form_lu(S, J, gamma, st);
    return newton_iter(S, J, C, h, Z, w, y, dy, st);
}

/* Corrector update of the history after an accepted step. */
static void correct(int nv, int q, const coef_t *C, double *Z, const double *y, const double *dy)
{
    const double *l = C->l;
    for (int i = 0; i < nv; i++) {
        double e = dy[i] / l[0];
        for (int j = 1; j <= q; j++) Z[(size_t)j * nv + i] += l[j] * e;
        Z[i] = y[i];
    }
}

int orc_burn_zone(const orc_net *net, double *row, const double *scale, double dt, double rtol,
                  double atol, int max_steps, orc_stats *st)
{
    return orc_burn_zone_ex(net, row, scale, NULL, dt, rtol, atol, max_steps, 0, 0, 0, st);
}

int orc_burn_zone_src(const orc_net *net, double *row, const double *scale, const double *src,
                      double dt, double rtol, double atol, int max_steps, orc_stats *st)
{
    return orc_burn_zone_ex(net, row, scale, src, dt, rtol, atol, max_steps, 0, 0, 0, st);
}

int orc_burn_zone_ex(const orc_net *net, double *row, const double *scale, const double *src,
                     double dt, double rtol, double atol, int max_steps, int jac_policy,
                     int fd_jac, int vc, orc_stats *st)
{
    sys_t S = {net, scale, orc_nvar(net), src};
    jac_t J;
    memset(&J, 0, sizeof J);
    J.policy = jac_policy;
    J.fd = fd_jac;
    J.rtol = rtol;
    J.atol = atol;
    int nv = S.nv;
    double Z[(ORC_QMAX + 2) * ORC_NVMAX], Zs[(ORC_QMAX + 2) * ORC_NVMAX];
    double w[ORC_NVMAX], f0[ORC_NVMAX], f1[ORC_NVMAX], y1[ORC_NVMAX];
    double y[ORC_NVMAX], dy[ORC_NVMAX], dyprev[ORC_NVMAX];
    memset(st, 0, sizeof(*st));
    memset(Z, 0, sizeof(Z));

    /* ---- start: Hairer-Norsett-Wanner step estimate for order 1 ---- */
    for (int i = 0; i < nv; i++) {
        if (!isfinite(row[i])) return ORC_NONFINITE;
        Z[i] = row[i];
        w[i] = atol + rtol * fabs(row[i]);
    }
    rhs(&S, Z, f0, st);
    for (int i = 0; i < nv; i++)
        if (!isfinite(f0[i])) return ORC_NONFINITE;
    double d0 = wrms(nv, Z, w), d1 = wrms(nv, f0, w);
    double ha = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    for (int i = 0; i < nv; i++) y1[i] = Z[i] + ha * f0[i];
    rhs(&S, y1, f1, st);
    for (int i = 0; i < nv; i++) dy[i] = f1[i] - f0[i];
    double d2 = wrms(nv, dy, w) / ha;
    double dm = fmax(d1, d2);
    double hb = (dm <= 1e-15) ? fmax(1e-6, ha * 1e-3) : sqrt(0.01 / dm);
    double h = fmin(fmin(100.0 * ha, hb), dt);
    if (!isfinite(h) || !(h > 0.0)) return ORC_NONFINITE;

    int q = 1, nequal = 0, nef = 0, ncf = 0, status = ORC_OK;
    double t = 0.0;
    for (int i = 0; i < nv; i++) { Z[nv + i] = h * f0[i]; dyprev[i] = 0.0; }
    double hist[ORC_QMAX];   /* accepted step sizes, newest first (variable-coefficient form) */
    int nh = 0;
    coef_t C;

    for (;;) {
        if (st->nst >= max_steps) { status = ORC_MAXSTEPS; break; }
        int last = 0;
        if (t + h >= dt * (1.0 - 4.0 * DBL_EPSILON)) {
            double eta = (dt - t) / h;
            rescale(nv, q, Z, eta);
            h = dt - t;
            nequal = 0;
            last = 1;
        }
        for (int i = 0; i < nv; i++) w[i] = atol + rtol * fabs(Z[i]);
        memcpy(Zs, Z, sizeof(double) * (size_t)(q + 1) * nv);
        predict(nv, q, Z);
        if (vc)
            coef_variable(q, h, hist, nh, &C);
        else
            coef_fixed(q, &C);

        if (newton(&S, &J, &C, h, Z, w, y, dy, st)) {
            memcpy(Z, Zs, sizeof(double) * (size_t)(q + 1) * nv);
            st->ncf++;
            if (++ncf >= 10) { status = ORC_CONV; break; }
            rescale(nv, q, Z, 0.25);
            h *= 0.25;
            nequal = 0;
            if (t + h == t) { status = ORC_HMIN; break; }
            continue;
        }

        double err = local_error(nv, &C, dy, w);
        /* Non-negativity (an inequality constraint on the abundances, as in CVODE): a step
           that takes a species below -atol is rejected like an error-test failure and cut
           to 0.9 of the fraction of it that keeps every species at or above -atol. */
        double feas = 1.0;
        for (int i = 0; i < net->ns && i < nv; i++) {
            if (y[i] < -atol) {
                double old = Zs[i];
                double frac = (old + atol) / (old - y[i]);
                feas = fmin(feas, frac);
            }
        }
        if (err > 1.0 || feas < 1.0) {
            memcpy(Z, Zs, sizeof(double) * (size_t)(q + 1) * nv);
            st->netf++;
            if (++nef >= 10) { status = ORC_ERRTEST; break; }
            double eta = err > 1.0 ? fmax(0.1, 1.0 / (pow(6.0 * err, 1.0 / (q + 1)) + 1e-6)) : 1.0;
            if (feas < 1.0) eta = fmin(eta, fmax(0.1, 0.9 * feas));
            if (nef >= 3) eta = 0.1;
            h *= eta;
            if (nef >= 3) {
                q = 1;
                nh = 0;      /* the restarted history is a tangent, not past values */
                rhs(&S, Z, f0, st);
                for (int i = 0; i < nv; i++) Z[nv + i] = h * f0[i];
            } else {
                rescale(nv, q, Z, eta);
            }
            nequal = 0;
            if (t + h == t) { status = ORC_HMIN; break; }
            continue;
        }

        /* ---- accept ---- */
        correct(nv, q, &C, Z, y, dy);
        for (int m = ORC_QMAX - 1; m > 0; m--) hist[m] = hist[m - 1];
        hist[0] = h;
        if (nh < ORC_QMAX) nh++;
        t = last ? dt : t + h;
        st->nst++;
        nequal++;
        nef = ncf = 0;
        if (last) break;

        if (nequal >= q + 1) {
            double best = 1.0 / (pow(6.0 * err, 1.0 / (q + 1)) + 1e-6);
            int qnew = q;
            if (q > 1) {
                double fact = 1.0;
                for (int i = 2; i <= q - 1; i++) fact *= i;
                double Em = fact * wrms(nv, Z + (size_t)q * nv, w);
                double etam = 1.0 / (pow(6.0 * Em, 1.0 / q) + 1e-6);
                if (etam > best) { best = etam; qnew = q - 1; }
            }
            if (q < ORC_QMAX) {
                double dd[ORC_NVMAX];
                for (int i = 0; i < nv; i++) dd[i] = dy[i] - dyprev[i];
                double Ep = wrms(nv, dd, w) / (q + 2);
                double etap = 1.0 / (pow(10.0 * Ep, 1.0 / (q + 2)) + 1e-6);
                if (etap > best) { best = etap; qnew = q + 1; }
            }
            if (best >= 1.5) {
                double eta = fmin(10.0, best);
                if (qnew == q + 1) {
                    orc_order_raise(nv, q, Z, dy);
                    q++;
                } else if (qnew == q - 1) {
                    orc_order_lower(nv, q, Z);
                    q--;
                }
                rescale(nv, q, Z, eta);
                h *= eta;
                nequal = 0;
            }
        }
        for (int i = 0; i < nv; i++) dyprev[i] = dy[i];
    }
    for (int i = 0; i < nv; i++) row[i] = Z[i];
    return status;
}

int orc_fixed_steps(const orc_net *net, const double *scale, int q, double h, int nsteps,
                    double *Zio, double *ys, double *errs)
{
    sys_t S = {net, scale, orc_nvar(net), NULL};
    int nv = S.nv;
    orc_stats st;
    jac_t J;
    memset(&J, 0, sizeof J);
    double Z[(ORC_QMAX + 2) * ORC_NVMAX], w[ORC_NVMAX], y[ORC_NVMAX], dy[ORC_NVMAX];
    memset(&st, 0, sizeof(st));
    memcpy(Z, Zio, sizeof(double) * (size_t)(q + 1) * nv);
    for (int n = 0; n < nsteps; n++) {
        for (int i = 0; i < nv; i++) w[i] = 1e-12 + 1e-8 * fabs(Z[i]);
        predict(nv, q, Z);
        coef_t C;
        coef_fixed(q, &C);
        if (newton(&S, &J, &C, h, Z, w, y, dy, &st)) return n + 1;
        if (errs) errs[n] = local_error(nv, &C, dy, w);
        correct(nv, q, &C, Z, y, dy);
        for (int i = 0; i < nv; i++) ys[(size_t)n * nv + i] = Z[i];
    }
    memcpy(Zio, Z, sizeof(double) * (size_t)(q + 1) * nv);
    return 0;
}

/* Fixed order q over the step sizes hs[0..nsteps) with the variable-coefficient form: Z (in
   units of hs[0]) is rescaled between steps, hist0 holds the nh0 past step sizes (newest
   first).  ys receives y after each step.  Returns 0, or 1 + the step whose Newton failed. */
int orc_vc_steps(const orc_net *net, const double *scale, int q, int nsteps, const double *hs,
                 const double *hist0, int nh0, double *Zio, double *ys)
{
    sys_t S = {net, scale, orc_nvar(net), NULL};
    int nv = S.nv;
    orc_stats st;
    jac_t J;
    memset(&J, 0, sizeof J);
    memset(&st, 0, sizeof st);
    double Z[(ORC_QMAX + 2) * ORC_NVMAX], w[ORC_NVMAX], y[ORC_NVMAX], dy[ORC_NVMAX];
    double hist[ORC_QMAX];
    int nh = nh0 < ORC_QMAX ? nh0 : ORC_QMAX;
    for (int m = 0; m < nh; m++) hist[m] = hist0[m];
    memcpy(Z, Zio, sizeof(double) * (size_t)(q + 1) * nv);
    for (int n = 0; n < nsteps; n++) {
        const double h = hs[n];
        if (n > 0) rescale(nv, q, Z, h / hs[n - 1]);
        for (int i = 0; i < nv; i++) w[i] = 1e-12 + 1e-8 * fabs(Z[i]);
        predict(nv, q, Z);
        coef_t C;
        coef_variable(q, h, hist, nh, &C);
        if (newton(&S, &J, &C, h, Z, w, y, dy, &st)) return n + 1;
        correct(nv, q, &C, Z, y, dy);
        for (int m = ORC_QMAX - 1; m > 0; m--) hist[m] = hist[m - 1];
        hist[0] = h;
        if (nh < ORC_QMAX) nh++;
        for (int i = 0; i < nv; i++) ys[(size_t)n * nv + i] = Z[i];
    }
    memcpy(Zio, Z, sizeof(double) * (size_t)(q + 1) * nv);
    return 0;
}

int orc_burn(const orc_net *net, double *state, int64_t zones, const double *scale, double dt,
             double rtol, double atol, int max_steps, int32_t *status, int32_t *stats, int nthreads)
{
    return orc_burn_src(net, state, zones, scale, NULL, dt, rtol, atol, max_steps, status, stats,
                        nthreads);
}

int orc_burn_src(const orc_net *net, double *state, int64_t zones, const double *scale,
                 const double *source, double dt, double rtol, double atol, int max_steps,
                 int32_t *status, int32_t *stats, int nthreads)
{
    return orc_burn_retry(net, state, zones, scale, source, dt, rtol, atol, max_steps, NULL, status,
                          stats, nthreads);
}

/* A failed zone (any status but ORC_OK) is integrated once more from its input with the
   retry tolerances, step cap and Jacobian (analytic, or finite differences) (the paper's
   zone-by-zone retry); success then reports
   ORC_OK_RETRY, a second failure that run's status.  Counters add up over both runs. */
int orc_burn_retry(const orc_net *net, double *state, int64_t zones, const double *scale,
                   const double *source, double dt, double rtol, double atol, int max_steps,
                   const orc_retry *retry, int32_t *status, int32_t *stats, int nthreads)
{
    return orc_burn_ex(net, state, zones, scale, source, dt, rtol, atol, max_steps, 0, 0, retry,
                       status, stats, nthreads);
}

int orc_burn_ex(const orc_net *net, double *state, int64_t zones, const double *scale,
                const double *source, double dt, double rtol, double atol, int max_steps,
                int jac_policy, int form, const orc_retry *retry, int32_t *status, int32_t *stats,
                int nthreads)
{
    if (orc_check_net(net)) return -1;
    int row = net->ns + 1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1) reduction(+ : bad)
    for (int64_t z = 0; z < zones; z++) {
        orc_stats st;
        double in[ORC_NVMAX + 1];
        double *y = state + z * row;
        const double *sc = scale ? scale + z * net->nr : NULL;
        const double *sr = source ? source + z * row : NULL;
        memcpy(in, y, sizeof(double) * row);
        int s = orc_burn_zone_ex(net, y, sc, sr, dt, rtol, atol, max_steps, jac_policy, 0, form, &st);
        if (s != ORC_OK && retry && retry->enabled) {
            orc_stats st2;
            memcpy(y, in, sizeof(double) * row);
            s = orc_burn_zone_ex(net, y, sc, sr, dt, retry->rtol, retry->atol, retry->max_steps,
                                 jac_policy, retry->jac, form, &st2);
            if (s == ORC_OK) s = ORC_OK_RETRY;
            st.nst += st2.nst; st.nfe += st2.nfe; st.nje += st2.nje; st.nlu += st2.nlu;
            st.nni += st2.nni; st.netf += st2.netf; st.ncf += st2.ncf;
        }
        if (status) status[z] = s;
        if (stats) memcpy(stats + z * 7, &st, sizeof(st));
        bad += (s != ORC_OK && s != ORC_OK_RETRY);
    }
    return bad;
}

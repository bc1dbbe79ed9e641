/*
 * Oracle RKC integrator (test infrastructure only; see oracle.h).
 *
 * The paper keeps the network separate from the integrator and names a
 * Runge-Kutta-Chebyshev method (Sommeijer, Shampine & Verwer 1998) beside
 * VODE, for zones that are only mildly stiff.  This file is the reading used
 * by the project, written from that paper's description of the method:
 *
 *  Scheme   The damped second-order RKC method with s >= 2 stages, damping
 *           eps = 2/13: w0 = 1 + eps/s^2, w1 = T_s'(w0)/T_s''(w0) (T_j the
 *           Chebyshev polynomials of the first kind), b_j = T_j''(w0)/T_j'(w0)^2
 *           for j >= 2 with b_0 = b_1 = b_2, a_j = 1 - b_j T_j(w0), and
 *             Y_0 = y_n,  Y_1 = Y_0 + mu~_1 h F(Y_0),  mu~_1 = b_1 w1,
 *             Y_j = (1 - mu_j - nu_j) Y_0 + mu_j Y_{j-1} + nu_j Y_{j-2}
 *                   + mu~_j h F(Y_{j-1}) + gamma~_j h F(Y_0),   j = 2..s,
 *           mu_j = 2 b_j w0 / b_{j-1}, nu_j = -b_j / b_{j-2},
 *           mu~_j = 2 b_j w1 / b_{j-1}, gamma~_j = -a_{j-1} mu~_j;
 *           y_{n+1} = Y_s.  (The networks are autonomous, so the stage times
 *           are not needed.)  On y' = lambda y one step multiplies y by
 *           a_s + b_s T_s(w0 + w1 h lambda).
 *  Stages   s = 1 + floor(sqrt(1 + 1.54 h rho)), at least 2, with rho the
 *           Gershgorin bound max_i sum_j |J_ij| of the analytic Jacobian at y_n
 *           (taken every step); h is first cut so that s <= 250.
 *  Error    est = (12 (y_n - y_{n+1}) + 6 h (F(y_n) + F(y_{n+1}))) / 15 in the
 *           weighted RMS norm with w_i = atol + rtol max(|y_n,i|, |y_{n+1},i|);
 *           a step is accepted when the norm is <= 1.
 *  Control  h *= min(10, max(0.1, 0.8 err^(-1/3))) after every step, accepted
 *           or not (the local error is O(h^3)).  The start (Hairer-Norsett-
 *           Wanner estimate), the landing on dt, the abundance constraint
 *           (a step that takes a species below -atol is rejected and cut to
 *           0.9 of its feasible fraction, at least 0.1) and the failure
 *           statuses are those of the BDF integrator; ten consecutive
 *           rejections end the zone with ERRTEST.
 *  Counters nst steps, nfe RHS evaluations, nje Jacobians, netf rejections.
 */
#include <float.h>
#include <math.h>
#include <string.h>

#include "oracle.h"

static double wrms_max(int nv, const double *v, const double *y0, const double *y1, double rtol,
                       double atol)
{
    double s = 0.0;
    for (int i = 0; i < nv; i++) {
        double w = atol + rtol * fmax(fabs(y0[i]), fabs(y1[i]));
        double x = v[i] / w;
        s += x * x;
    }
    return sqrt(s / nv);
}

static double wrms_w(int nv, const double *v, const double *w)
{
    double s = 0.0;
    for (int i = 0; i < nv; i++) {
        double x = v[i] / w[i];
        s += x * x;
    }
    return sqrt(s / nv);
}

static void f_src(const orc_net *net, const double *scale, const double *src, int nv, const double *y,
                  double *f, orc_stats *st)
{
    orc_rhs(net, scale, y, f);
    if (src)
        for (int i = 0; i < nv; i++) f[i] += src[i];
    st->nfe++;
}

/* Gershgorin bound of the spectral radius of J at y. */
static double spectral_bound(const orc_net *net, const double *scale, int nv, const double *y,
                             orc_stats *st)
{
    double J[ORC_NVMAX * ORC_NVMAX];
    orc_jac(net, scale, y, J);
    st->nje++;
    double rho = 0.0;
    for (int i = 0; i < nv; i++) {
        double r = 0.0;
        for (int j = 0; j < nv; j++) r += fabs(J[i * nv + j]);
        rho = fmax(rho, r);
    }
    return rho;
}

/* Number of stages for step h: s = 1 + floor(sqrt(1 + 1.54 h rho)), at least 2. */
int orc_rkc_stages(double h, double rho)
{
    int s = 1 + (int)floor(sqrt(1.0 + 1.54 * h * rho));
    return s < 2 ? 2 : s;
}

/* One RKC step of s stages from y0 (f0 = F(y0)); writes y1.  Uses s - 1 further RHS calls. */
static void rkc_step(const orc_net *net, const double *scale, const double *src, int nv, int s,
                     double h, const double *y0, const double *f0, double *y1, orc_stats *st)
{
    const double eps = 2.0 / 13.0;
    const double w0 = 1.0 + eps / ((double)s * s);
    double T[ORC_RKC_SMAX + 1], dT[ORC_RKC_SMAX + 1], ddT[ORC_RKC_SMAX + 1];
    T[0] = 1.0; T[1] = w0;
    dT[0] = 0.0; dT[1] = 1.0;
    ddT[0] = 0.0; ddT[1] = 0.0;
    /* s >= 2: the j = 2 terms always exist */
    T[2] = 2.0 * w0 * T[1] - T[0];
    dT[2] = 2.0 * T[1] + 2.0 * w0 * dT[1] - dT[0];
    ddT[2] = 4.0 * dT[1] + 2.0 * w0 * ddT[1] - ddT[0];
    for (int j = 3; j <= s; j++) {
        T[j] = 2.0 * w0 * T[j - 1] - T[j - 2];
        dT[j] = 2.0 * T[j - 1] + 2.0 * w0 * dT[j - 1] - dT[j - 2];
        ddT[j] = 4.0 * dT[j - 1] + 2.0 * w0 * ddT[j - 1] - ddT[j - 2];
    }
    const double w1 = dT[s] / ddT[s];
    double b[ORC_RKC_SMAX + 1];
    b[2] = ddT[2] / (dT[2] * dT[2]);
    for (int j = 3; j <= s; j++) b[j] = ddT[j] / (dT[j] * dT[j]);
    b[0] = b[1] = b[2];

    double Yjm2[ORC_NVMAX], Yjm1[ORC_NVMAX], Yj[ORC_NVMAX], F[ORC_NVMAX];
    for (int i = 0; i < nv; i++) {
        Yjm2[i] = y0[i];
        Yjm1[i] = y0[i] + b[1] * w1 * h * f0[i];
    }
    for (int j = 2; j <= s; j++) {
        const double mu = 2.0 * b[j] * w0 / b[j - 1];
        const double nu = -b[j] / b[j - 2];
        const double mut = 2.0 * b[j] * w1 / b[j - 1];
        const double gat = -(1.0 - b[j - 1] * T[j - 1]) * mut;
        f_src(net, scale, src, nv, Yjm1, F, st);
        for (int i = 0; i < nv; i++)
            Yj[i] = (1.0 - mu - nu) * y0[i] + mu * Yjm1[i] + nu * Yjm2[i] + mut * h * F[i] + gat * h * f0[i];
        memcpy(Yjm2, Yjm1, sizeof(double) * nv);
        memcpy(Yjm1, Yj, sizeof(double) * nv);
    }
    memcpy(y1, Yjm1, sizeof(double) * nv);
}

int orc_rkc_fixed(const orc_net *net, const double *scale, double *y, double h, int nsteps, int s)
{
    int nv = orc_nvar(net);
    if (s < 2 || s > ORC_RKC_SMAX) return -1;
    orc_stats st;
    memset(&st, 0, sizeof st);
    double f0[ORC_NVMAX], y1[ORC_NVMAX];
    for (int n = 0; n < nsteps; n++) {
        f_src(net, scale, NULL, nv, y, f0, &st);
        rkc_step(net, scale, NULL, nv, s, h, y, f0, y1, &st);
        memcpy(y, y1, sizeof(double) * nv);
    }
    return 0;
}

int orc_rkc_zone(const orc_net *net, double *row, const double *scale, const double *src, double dt,
                 double rtol, double atol, int max_steps, orc_stats *st)
{
    const int nv = orc_nvar(net);
    double y[ORC_NVMAX], f0[ORC_NVMAX], y1[ORC_NVMAX], f1[ORC_NVMAX], w[ORC_NVMAX], est[ORC_NVMAX];
    memset(st, 0, sizeof(*st));
    for (int i = 0; i < nv; i++) {
        if (!isfinite(row[i]) || (src && !isfinite(src[i]))) return ORC_NONFINITE;
        y[i] = row[i];
        w[i] = atol + rtol * fabs(row[i]);
    }
    /* start: the Hairer-Norsett-Wanner estimate, as for the BDF integrator */
    f_src(net, scale, src, nv, y, f0, st);
    for (int i = 0; i < nv; i++)
        if (!isfinite(f0[i])) return ORC_NONFINITE;
    double d0 = wrms_w(nv, y, w), d1 = wrms_w(nv, f0, w);
    double ha = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    for (int i = 0; i < nv; i++) y1[i] = y[i] + ha * f0[i];
    f_src(net, scale, src, nv, y1, f1, st);
    for (int i = 0; i < nv; i++) est[i] = f1[i] - f0[i];
    double d2 = wrms_w(nv, est, w) / ha;
    double dm = fmax(d1, d2);
    double hb = (dm <= 1e-15) ? fmax(1e-6, ha * 1e-3) : sqrt(0.01 / dm);
    double h = fmin(fmin(100.0 * ha, hb), dt);
    if (!isfinite(h) || !(h > 0.0)) return ORC_NONFINITE;

    double t = 0.0;
    int nrej = 0;
    for (;;) {
        if (st->nst >= max_steps) { for (int i = 0; i < nv; i++) row[i] = y[i]; return ORC_MAXSTEPS; }
        int last = 0;
        if (t + h >= dt * (1.0 - 4.0 * DBL_EPSILON)) {
            h = dt - t;
            last = 1;
        }
        const double rho = spectral_bound(net, scale, nv, y, st);
        const double hstab = ((double)(ORC_RKC_SMAX - 1) * (ORC_RKC_SMAX - 1) - 1.0) / (1.54 * rho);
        if (h > hstab) {
            h = hstab;
            last = 0;
        }
        const int s = orc_rkc_stages(h, rho);
        rkc_step(net, scale, src, nv, s, h, y, f0, y1, st);
        f_src(net, scale, src, nv, y1, f1, st);
        for (int i = 0; i < nv; i++) est[i] = (12.0 * (y[i] - y1[i]) + 6.0 * h * (f0[i] + f1[i])) / 15.0;
        double err = wrms_max(nv, est, y, y1, rtol, atol);
        double feas = 1.0;
        for (int i = 0; i < net->ns && i < nv; i++)
            if (y1[i] < -atol) feas = fmin(feas, (y[i] + atol) / (y[i] - y1[i]));
        if (!isfinite(err)) err = 1e10;
        double fac = fmin(10.0, fmax(0.1, 0.8 * pow(err, -1.0 / 3.0)));
        if (err > 1.0 || feas < 1.0) {
            st->netf++;
            if (++nrej >= 10) { for (int i = 0; i < nv; i++) row[i] = y[i]; return ORC_ERRTEST; }
            if (feas < 1.0) fac = fmin(fac, fmax(0.1, 0.9 * feas));
            h *= fmin(fac, 1.0);
            if (t + h == t) { for (int i = 0; i < nv; i++) row[i] = y[i]; return ORC_HMIN; }
            continue;
        }
        /* accept */
        nrej = 0;
        memcpy(y, y1, sizeof(double) * nv);
        memcpy(f0, f1, sizeof(double) * nv);
        t = last ? dt : t + h;
        st->nst++;
        if (last) break;
        h *= fac;
    }
    for (int i = 0; i < nv; i++) row[i] = y[i];
    return ORC_OK;
}

int orc_rkc(const orc_net *net, double *state, int64_t zones, const double *scale, const double *source,
            double dt, double rtol, double atol, int max_steps, int32_t *status, int32_t *stats,
            int nthreads)
{
    if (orc_check_net(net)) return -1;
    int row = net->ns + 1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1) reduction(+ : bad)
    for (int64_t z = 0; z < zones; z++) {
        orc_stats st;
        int s = orc_rkc_zone(net, state + z * row, scale ? scale + z * net->nr : NULL,
                             source ? source + z * row : NULL, dt, rtol, atol, max_steps, &st);
        if (status) status[z] = s;
        if (stats) memcpy(stats + z * 7, &st, sizeof(st));
        bad += (s != ORC_OK);
    }
    return bad;
}

/*
 * Brute-force reference integrator (test infrastructure only; see oracle.h).
 *
 * Two-stage Radau IIA (order 3, L-stable): c = (1/3, 1),
 * A = [[5/12, -1/12], [3/4, 1/4]], y_{n+1} = Y_2.  Fixed steps on a geometric
 * mesh whose first step is h0 (uniform when h0 <= 0), and for every step a full
 * Newton iteration (Jacobian re-evaluated at every iterate) on the 2 nv stage
 * equations, run to rounding level.  Nothing here is shared with the BDF code:
 * it is an independent method used to check the BDF results on tiny batches.
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

static double mesh_ratio(double dt, int64_t n, double h0)
{
    /* h0 (r^n - 1) / (r - 1) = dt, r > 1, by bisection on log r */
    double lo = 0.0, hi = 50.0 / (double)n + 1.0;
    for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi);
        double r = exp(mid);
        double s = h0 * expm1((double)n * mid) / (r - 1.0);
        if (s > dt) hi = mid; else lo = mid;
    }
    return exp(0.5 * (lo + hi));
}

int orc_radau(const orc_net *net, const double *scale, double *y, double dt, int64_t nsteps, double h0)
{
    const double a11 = 5.0 / 12.0, a12 = -1.0 / 12.0, a21 = 3.0 / 4.0, a22 = 1.0 / 4.0;
    int nv = orc_nvar(net);
    int n2 = 2 * nv;
    double r = 1.0;
    int geometric = (h0 > 0.0 && h0 * (double)nsteps < dt);
    if (geometric) r = mesh_ratio(dt, nsteps, h0);
    else h0 = dt / (double)nsteps;

    double Y1[ORC_NVMAX], Y2[ORC_NVMAX], F1[ORC_NVMAX], F2[ORC_NVMAX];
    double J1[ORC_NVMAX * ORC_NVMAX], J2[ORC_NVMAX * ORC_NVMAX];
    static _Thread_local double A[4 * ORC_NVMAX * ORC_NVMAX];
    double g[2 * ORC_NVMAX];
    int piv[2 * ORC_NVMAX];

    double t = 0.0, h = h0;
    for (int64_t n = 0; n < nsteps; n++) {
        if (n == nsteps - 1) h = dt - t;
        memcpy(Y1, y, sizeof(double) * nv);
        memcpy(Y2, y, sizeof(double) * nv);
        double prev = INFINITY;
        int ok = 0;
        for (int it = 0; it < 60; it++) {
            orc_rhs(net, scale, Y1, F1);
            orc_rhs(net, scale, Y2, F2);
            orc_jac(net, scale, Y1, J1);
            orc_jac(net, scale, Y2, J2);
            for (int i = 0; i < nv; i++) {
                g[i] = -(Y1[i] - y[i] - h * (a11 * F1[i] + a12 * F2[i]));
                g[nv + i] = -(Y2[i] - y[i] - h * (a21 * F1[i] + a22 * F2[i]));
            }
            for (int i = 0; i < nv; i++) {
                for (int j = 0; j < nv; j++) {
                    double e = (i == j) ? 1.0 : 0.0;
                    A[i * n2 + j] = e - h * a11 * J1[i * nv + j];
                    A[i * n2 + nv + j] = -h * a12 * J2[i * nv + j];
                    A[(nv + i) * n2 + j] = -h * a21 * J1[i * nv + j];
                    A[(nv + i) * n2 + nv + j] = e - h * a22 * J2[i * nv + j];
                }
            }
            if (orc_lu(n2, A, piv)) return -(int)(n + 1);
            orc_lu_solve(n2, A, piv, g);
            double dn = 0.0, yn = 0.0;
            for (int i = 0; i < nv; i++) {
                Y1[i] += g[i];
                Y2[i] += g[nv + i];
                dn = fmax(dn, fmax(fabs(g[i]), fabs(g[nv + i])));
                yn = fmax(yn, fmax(fabs(Y1[i]), fabs(Y2[i])));
            }
            if (!isfinite(dn)) return -(int)(n + 1);
            if (dn <= 4e-16 * yn || (dn >= prev && dn <= 1e-12 * yn)) { ok = 1; break; }
            prev = dn;
        }
        if (!ok) return -(int)(n + 1);
        memcpy(y, Y2, sizeof(double) * nv);
        t += h;
        h *= r;
    }
    return 0;
}

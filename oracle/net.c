/*
 * Oracle network evaluation (test infrastructure only; see oracle.h).
 *
 * Mass-action kinetics with Arrhenius rates.  For reaction r with reactants
 * a (and b, if second order) and products c (and d):
 *   k_r = s_r * exp(lnA_r + n_r ln T - E_r / T)        (thermal network)
 *   k_r = s_r * exp(lnA_r)                             (no temperature coupling)
 *   w_r = s_r k_r Y_a Y_b (k_r Y_a for a first-order reaction), where the sign
 *         s_r = -1 when both reactants are negative and +1 otherwise; for
 *         A + A this is k Y_A |Y_A|.
 * The exact solution never leaves Y >= 0, where s_r = 1 and this is plain mass
 * action.  Off that set the sign makes a negative abundance be pulled back to
 * zero, as one negative reactant with a positive partner already is, instead
 * of running away: with s_r = 1 a quadratic self-reaction gives dY/dt = -2k Y^2,
 * which diverges for Y < 0.  w stays continuous, and for A + A continuously
 * differentiable; mass is conserved exactly.
 *   dY_i/dt = sum_r nu_ir w_r,   nu_ir = #(i among products) - #(i among reactants)
 *   dT/dt   = sum_r q_r w_r      (thermal network only)
 * The Jacobian is the exact derivative of this right-hand side.
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

int orc_nvar(const orc_net *net) { return net->ns + (net->thermal ? 1 : 0); }

int orc_check_net(const orc_net *net)
{
    if (net->ns < 1 || net->nr < 0 || orc_nvar(net) > ORC_NVMAX) return 1;
    for (int r = 0; r < net->nr; r++) {
        int a = net->reactant[2 * r], b = net->reactant[2 * r + 1];
        int c = net->product[2 * r], d = net->product[2 * r + 1];
        if (a < 0 || a >= net->ns || b < -1 || b >= net->ns) return 1;
        if (c < 0 || c >= net->ns || d < -1 || d >= net->ns) return 1;
    }
    return 0;
}

void orc_rates(const orc_net *net, const double *scale, const double *y, double *k, double *dkdT)
{
    double T = net->thermal ? y[net->ns] : 0.0;
    for (int r = 0; r < net->nr; r++) {
        double s = scale ? scale[r] : 1.0;
        if (net->thermal) {
            double arg = net->lnA[r] + net->n_exp[r] * log(T) - net->E[r] / T;
            k[r] = s * exp(arg);
            if (dkdT) dkdT[r] = k[r] * (net->n_exp[r] + net->E[r] / T) / T;
        } else {
            k[r] = s * exp(net->lnA[r]);
            if (dkdT) dkdT[r] = 0.0;
        }
    }
}

void orc_rhs(const orc_net *net, const double *scale, const double *y, double *f)
{
    int nv = orc_nvar(net);
    double k[4096];
    for (int i = 0; i < nv; i++) f[i] = 0.0;
    orc_rates(net, scale, y, k, NULL);
    for (int r = 0; r < net->nr; r++) {
        int a = net->reactant[2 * r], b = net->reactant[2 * r + 1];
        int c = net->product[2 * r], d = net->product[2 * r + 1];
        double w = k[r] * y[a];
        if (b >= 0) w *= (y[a] < 0.0 && y[b] < 0.0) ? -y[b] : y[b];
        f[a] -= w;
        if (b >= 0) f[b] -= w;
        f[c] += w;
        if (d >= 0) f[d] += w;
        if (net->thermal) f[net->ns] += net->q[r] * w;
    }
}

/* Same right-hand side in complex arithmetic, for complex-step derivative checks. */
void orc_rhs_cplx(const orc_net *net, const double *scale, const double complex *y, double complex *f)
{
    int nv = orc_nvar(net);
    for (int i = 0; i < nv; i++) f[i] = 0.0;
    for (int r = 0; r < net->nr; r++) {
        double s = scale ? scale[r] : 1.0;
        double complex kr;
        if (net->thermal) {
            double complex T = y[net->ns];
            kr = s * cexp(net->lnA[r] + net->n_exp[r] * clog(T) - net->E[r] / T);
        } else {
            kr = s * exp(net->lnA[r]);
        }
        int a = net->reactant[2 * r], b = net->reactant[2 * r + 1];
        int c = net->product[2 * r], d = net->product[2 * r + 1];
        double complex w = kr * y[a];
        if (b >= 0) w *= (creal(y[a]) < 0.0 && creal(y[b]) < 0.0) ? -y[b] : y[b];
        f[a] -= w;
        if (b >= 0) f[b] -= w;
        f[c] += w;
        if (d >= 0) f[d] += w;
        if (net->thermal) f[net->ns] += net->q[r] * w;
    }
}

void orc_jac(const orc_net *net, const double *scale, const double *y, double *J)
{
    int nv = orc_nvar(net);
    double k[4096], dk[4096];
    memset(J, 0, sizeof(double) * nv * nv);
    orc_rates(net, scale, y, k, dk);
    for (int r = 0; r < net->nr; r++) {
        int a = net->reactant[2 * r], b = net->reactant[2 * r + 1];
        int c = net->product[2 * r], d = net->product[2 * r + 1];
        /* partial derivatives of w_r */
        double dwa, dwb = 0.0, dwT = 0.0;
        if (b >= 0) {
            double sg = (y[a] < 0.0 && y[b] < 0.0) ? -1.0 : 1.0;
            dwa = sg * k[r] * y[b];
            dwb = sg * k[r] * y[a];
            if (net->thermal) dwT = sg * dk[r] * y[a] * y[b];
        } else {
            dwa = k[r];
            if (net->thermal) dwT = dk[r] * y[a];
        }
        /* rows touched by reaction r and their stoichiometric weights */
        int rows[5];
        double wt[5];
        int nrow = 0;
        rows[nrow] = a; wt[nrow++] = -1.0;
        if (b >= 0) { rows[nrow] = b; wt[nrow++] = -1.0; }
        rows[nrow] = c; wt[nrow++] = 1.0;
        if (d >= 0) { rows[nrow] = d; wt[nrow++] = 1.0; }
        if (net->thermal) { rows[nrow] = net->ns; wt[nrow++] = net->q[r]; }
        for (int m = 0; m < nrow; m++) {
            double *Jrow = J + (size_t)rows[m] * nv;
            Jrow[a] += wt[m] * dwa;
            if (b >= 0) Jrow[b] += wt[m] * dwb;
            if (net->thermal) Jrow[net->ns] += wt[m] * dwT;
        }
    }
}

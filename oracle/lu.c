/*
 * Oracle dense linear algebra (test infrastructure only; see oracle.h).
 *
 * Gaussian elimination with partial (row) pivoting, textbook form: at step k
 * the pivot is the entry of largest magnitude in column k on or below the
 * diagonal, the first such row on ties; rows are exchanged explicitly and the
 * multipliers overwrite the eliminated entries, so A holds L (unit lower,
 * below the diagonal) and U (on and above it) of P A = L U.
 */
#include <math.h>

#include "oracle.h"

int orc_lu(int n, double *A, int *piv)
{
    int info = 0;
    for (int k = 0; k < n; k++) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; i++) {
            double v = fabs(A[i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (p != k) {
            for (int j = 0; j < n; j++) {
                double t = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = t;
            }
        }
        double pv = A[k * n + k];
        if (pv == 0.0) {
            if (!info) info = k + 1;
            continue;
        }
        for (int i = k + 1; i < n; i++) {
            double l = A[i * n + k] / pv;
            A[i * n + k] = l;
            for (int j = k + 1; j < n; j++) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return info;
}

void orc_lu_solve(int n, const double *LU, const int *piv, double *b)
{
    for (int k = 0; k < n; k++) {
        int p = piv[k];
        if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
    }
    for (int i = 1; i < n; i++) {
        double s = b[i];
        for (int j = 0; j < i; j++) s -= LU[i * n + j] * b[j];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = b[i];
        for (int j = i + 1; j < n; j++) s -= LU[i * n + j] * b[j];
        b[i] = s / LU[i * n + i];
    }
}

/*
 * Oracle step O6: banded LU factorisation WITHOUT pivoting and the two
 * triangular solves, complex128, plain loops.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by oracle/band.py; nothing in the product
 * links or calls this file.
 *
 * The paper does not name its local solver; its Table 4 splits a one-off
 * "setup" phase from the iterations, which is read as: every local operator
 * A_j is factorised once and reused by every preconditioner application
 * (Section 2, B^{-1} = sum_j R~_j^T A_j^{-1} R_j).  The oracle factorises
 * A = L U with L unit lower triangular and U upper triangular (Doolittle),
 * no row exchanges.  When it exists this factorisation is unique.
 *
 * Storage: row r of the band occupies AB[r*(2b+1) .. r*(2b+1)+2b], and
 * entry (r, c) with |r - c| <= b sits at AB[r*(2b+1) + b + (c - r)].
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>

typedef double complex zc;

#define AT(AB, w, b, r, c) (AB)[(size_t)(r) * (size_t)(w) + (size_t)((b) + (c) - (r))]

/* Returns 0, or 1 + the column whose pivot magnitude is <= tol_abs. */
int oracle_band_lu(int n, int b, zc *AB, double tol_abs, double *max_u)
{
    const int w = 2 * b + 1;
    double mu = 0.0;
    for (int c = 0; c < n; ++c) {
        zc piv = AT(AB, w, b, c, c);
        if (cabs(piv) <= tol_abs) {
            if (max_u) *max_u = mu;
            return c + 1;
        }
        int last = c + b < n - 1 ? c + b : n - 1;
        for (int r = c + 1; r <= last; ++r) {
            zc l = AT(AB, w, b, r, c) / piv;
            AT(AB, w, b, r, c) = l;
            if (l == 0.0) continue;
            for (int cc = c + 1; cc <= last; ++cc)
                AT(AB, w, b, r, cc) -= l * AT(AB, w, b, c, cc);
        }
        for (int cc = c; cc <= last; ++cc) {
            double a = cabs(AT(AB, w, b, c, cc));
            if (a > mu) mu = a;
        }
    }
    if (max_u) *max_u = mu;
    return 0;
}

/* x <- U^{-1} L^{-1} x using the factors written by oracle_band_lu. */
void oracle_band_solve(int n, int b, const zc *LU, zc *x)
{
    const int w = 2 * b + 1;
    for (int r = 0; r < n; ++r) {                 /* L y = x, L unit lower */
        zc s = x[r];
        int first = r - b > 0 ? r - b : 0;
        for (int c = first; c < r; ++c) s -= AT(LU, w, b, r, c) * x[c];
        x[r] = s;
    }
    for (int r = n - 1; r >= 0; --r) {            /* U x = y */
        zc s = x[r];
        int last = r + b < n - 1 ? r + b : n - 1;
        for (int c = r + 1; c <= last; ++c) s -= AT(LU, w, b, r, c) * x[c];
        x[r] = s / AT(LU, w, b, r, r);
    }
}

/* Batched drivers: matrix m has size n[m], half-bandwidth b[m], and its band
 * array starts at element off[m] of data; vector m starts at voff[m]. */
void oracle_band_lu_batch(int nm, const int *n, const int *b, const long long *off,
                          zc *data, const double *tol_abs, int *status, double *max_u,
                          int nthreads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int m = 0; m < nm; ++m)
        status[m] = oracle_band_lu(n[m], b[m], data + off[m], tol_abs[m], max_u + m);
}

void oracle_band_solve_batch(int nm, const int *n, const int *b, const long long *off,
                             const zc *data, const long long *voff, zc *vec, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int m = 0; m < nm; ++m)
        oracle_band_solve(n[m], b[m], data + off[m], vec + voff[m]);
}

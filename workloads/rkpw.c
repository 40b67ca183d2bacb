/*
 * Reconstruction of a symmetric tridiagonal (Jacobi) matrix from prescribed
 * eigenvalues and the first components of its eigenvectors.
 *
 * This is an input generator, not part of any eigensolver.  Running n steps of
 * Lanczos on diag(lam) from the unit start vector w yields the tridiagonal
 * T = Q^T diag(lam) Q with Q e_1 = w.  Plain Lanczos loses orthogonality, and
 * full reorthogonalisation costs O(n^3), so the same T is built here by the
 * numerically stable O(n^2) rotation scheme of Rutishauser / Gragg-Harrod:
 * the bordered matrix [[0, w^T], [w, diag(lam)]] is reduced to tridiagonal form
 * by inserting one (lam_m, w_m) pair at a time and chasing the bulge that each
 * insertion creates down the band with Givens rotations.
 *
 * On return alpha[0..n-1] is the diagonal and beta[0..n-2] the (non-negative)
 * off-diagonal of T.  Returns 0 on success, -1 on bad arguments.
 */
#include <math.h>
#include <stddef.h>

int wl_rkpw(int n, const double *lam, const double *w, double *alpha, double *beta)
{
    if (n < 0 || (n > 0 && (!lam || !w || !alpha || (n > 1 && !beta))))
        return -1;
    if (n == 0)
        return 0;
    double b0 = 0.0; /* coupling of the border row to the first band index */
    int k = 0;       /* current band size */
    for (int m = 0; m < n; ++m) {
        const double lm = lam[m], om = w[m];
        if (k == 0) {
            alpha[0] = lm;
            b0 = fabs(om);
            k = 1;
            continue;
        }
        /* Index order before the chase: border, new x, t0, t1, ..., t_{k-1}.
         * p is the last finished index, u the pending one, v the next band
         * index.  f = p-u coupling, g = p-v coupling (to be annihilated),
         * du = u diagonal, h = u-v coupling. */
        double f = om, g = b0, du = lm, h = 0.0;
        for (int j = 0; j < k; ++j) {
            const double dv = alpha[j];
            const double r = hypot(f, g);
            double c = 1.0, s = 0.0;
            if (r != 0.0) {
                c = f / r;
                s = g / r;
            }
            if (j == 0)
                b0 = r;
            else
                beta[j - 1] = r;
            const double uu = c * c * du + 2.0 * c * s * h + s * s * dv;
            const double vv = s * s * du - 2.0 * c * s * h + c * c * dv;
            const double uv = c * s * (dv - du) + (c * c - s * s) * h;
            alpha[j] = uu;
            const double bj = (j < k - 1) ? beta[j] : 0.0;
            f = uv;
            g = s * bj;
            du = vv;
            h = c * bj;
        }
        alpha[k] = du;
        beta[k - 1] = f;
        ++k;
    }
    for (int i = 0; i + 1 < n; ++i)
        beta[i] = fabs(beta[i]);
    return 0;
}

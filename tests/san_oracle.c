/* Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (oracle/oracle.c): eigenvalues, eigenvectors, counts, the norm and
 * the double-double primitives on small matrices of the kinds the tests use
 * (random, 1-2-1, glued blocks with tiny couplings, a split matrix, n = 1 and
 * 2).  Any invalid access or undefined operation aborts the run. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_eigvals(int n, const double *d, const double *e, int il, int iu, double *w_hi,
                   double *w_lo, int threads);
int oracle_count(int n, const double *d, const double *e, double sig_hi, double sig_lo);
int oracle_eigvecs(int n, const double *d, const double *e, int m, const double *w_hi,
                   const double *w_lo, double *z, unsigned long long seed, double group_tol,
                   int threads);
double oracle_tnorm(int n, const double *d, const double *e);
void oracle_dd_op(int op, double ah, double al, double bh, double bl, double *rh, double *rl);

static unsigned long long st = 88172645463325252ull;
static double urand(void) {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return (double)(st >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static int run(int n, const double *d, const double *e) {
    double *wh = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *wl = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *z = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (n > 0 ? n : 1));
    int rc = oracle_eigvals(n, d, e, 1, n, wh, wl, 2);
    if (!rc) rc = oracle_eigvecs(n, d, e, n, wh, wl, z, 12345ull, 0.0, 2);
    if (!rc && n > 2) rc = oracle_eigvals(n, d, e, 2, n - 1, wh, wl, 1);
    if (!rc && n > 0) {
        const int c = oracle_count(n, d, e, 0.0, 0.0);
        if (c < 0 || c > n) rc = 1;
    }
    (void)oracle_tnorm(n, d, e);
    free(wh);
    free(wl);
    free(z);
    return rc;
}

int main(void) {
    int bad = 0;
    for (int n = 1; n <= 40; n += 13) {
        double d[64], e[64];
        for (int i = 0; i < n; ++i) d[i] = urand();
        for (int i = 0; i + 1 < n; ++i) e[i] = urand();
        e[n > 1 ? n - 1 : 0] = 0.0;
        bad |= run(n, d, e);
        for (int i = 0; i < n; ++i) d[i] = 2.0;
        for (int i = 0; i + 1 < n; ++i) e[i] = 1.0;
        bad |= run(n, d, e);
        for (int i = 0; i < n; ++i) d[i] = fabs(10.0 - (double)(i % 21));
        for (int i = 0; i + 1 < n; ++i) e[i] = ((i + 1) % 21 == 0) ? 1e-10 : 1.0;
        bad |= run(n, d, e);
        if (n > 5) {
            e[2] = 0.0;  /* split */
            bad |= run(n, d, e);
        }
    }
    double rh, rl;
    for (int op = 0; op < 5; ++op) oracle_dd_op(op, 1.5, 1e-17, -0.75, 3e-18, &rh, &rl);
    printf(bad ? "oracle sanitizer run: FAILED\n" : "oracle sanitizer run: ok\n");
    return bad;
}

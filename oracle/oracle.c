/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow CPU solver for the real symmetric tridiagonal eigenproblem
 * T z = lambda z (the problem statement of the paper's introduction): the
 * i-th smallest eigenvalue of T and a unit eigenvector, for an index range
 * il..iu.  It is the reference the HIP path is checked against and shares no
 * code with it.  Only the test-suite, the smoke check and the benchmark's CPU
 * baseline may use it.
 *
 * Method (a different textbook method from the one under test, carried out in
 * double-double so that its own error is far below the I/O precision):
 *   1. the FP32/FP64 input is promoted exactly to double-double and scaled
 *      by a power of two so that ||T||_1 lies in [1/2, 1) (the scaling of the
 *      entries in the paper's preprocessing; exact, and undone on output);
 *   2. eigenvalue i by bisection on the Sturm count of T - sigma I, i.e. the
 *      number of negative pivots of its LDL^T (Sylvester inertia), evaluated
 *      with the classic recurrence q_1 = d_1 - sigma,
 *      q_j = (d_j - sigma) - e_{j-1}^2 / q_{j-1};
 *   3. eigenvector i by inverse iteration with (T - lambda_i I), solved by
 *      Gaussian elimination with partial pivoting, from a seeded start vector;
 *      eigenvalues that coincide to within 2^-60 ||T||_1 form a group whose
 *      vectors are made orthogonal by modified Gram-Schmidt after each step;
 *   4. each vector is normalised and signed so that its largest-magnitude
 *      entry is positive.
 * No splitting, no shifting and no perturbation of T is done.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int omp_threads(void) { return omp_get_max_threads(); }

/* ORACLE_MUTANT selects a deliberately wrong variant (0 = the real oracle).
 * The pin tests compile each mutant and check that some pin rejects it. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

/* ------------------------------------------------------------------------ */
/* double-double arithmetic (Dekker / Knuth error-free transformations)       */
/* ------------------------------------------------------------------------ */
typedef struct {
    double hi, lo;
} xdd;

static xdd mk(double hi, double lo) { xdd r; r.hi = hi; r.lo = lo; return r; }
static xdd from_d(double a) { return mk(a, 0.0); }

/* exact a + b = s + err (Knuth) */
static xdd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double err = (a - (s - bb)) + (b - bb);
    return mk(s, err);
}
/* exact a + b when |a| >= |b| */
static xdd quick_two_sum(double a, double b)
{
    double s = a + b;
    return mk(s, b - (s - a));
}
/* exact a * b = p + err using a fused multiply-add */
static xdd two_prod(double a, double b)
{
    double p = a * b;
    return mk(p, fma(a, b, -p));
}
static xdd x_add(xdd a, xdd b)
{
    xdd s = two_sum(a.hi, b.hi);
    xdd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
static xdd x_neg(xdd a) { return mk(-a.hi, -a.lo); }
static xdd x_sub(xdd a, xdd b) { return x_add(a, x_neg(b)); }
static xdd x_mul(xdd a, xdd b)
{
    xdd p = two_prod(a.hi, b.hi);
    p.lo += (ORACLE_MUTANT == 4) ? a.hi * b.lo : a.hi * b.lo + a.lo * b.hi; /* mutant 4 drops a term */
    return quick_two_sum(p.hi, p.lo);
}
static xdd x_mul_d(xdd a, double b)
{
    xdd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
/* long division: three quotient digits, each corrected by the exact remainder */
static xdd x_div(xdd a, xdd b)
{
    double q1 = a.hi / b.hi;
    xdd r = x_sub(a, x_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = x_sub(r, x_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    xdd q = quick_two_sum(q1, q2);
    return x_add(q, from_d(q3));
}
static xdd x_sqrt(xdd a)
{
    if (a.hi <= 0.0)
        return from_d(0.0);
    double x = 1.0 / sqrt(a.hi);
    double ax = a.hi * x;
    /* one Newton step on the square root (Karp's trick) */
    xdd axx = x_mul(from_d(ax), from_d(ax));
    double corr = x_sub(a, axx).hi * (x * 0.5);
    return two_sum(ax, corr);
}
static int x_lt(xdd a, xdd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
static int x_eq(xdd a, xdd b) { return a.hi == b.hi && a.lo == b.lo; }
static xdd x_abs(xdd a) { return (a.hi < 0.0 || (a.hi == 0.0 && a.lo < 0.0)) ? x_neg(a) : a; }
static double x_to_d(xdd a) { return a.hi + a.lo; }

/* ------------------------------------------------------------------------ */
/* problem data                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    xdd *d;   /* diagonal, exact copy of the input */
    xdd *e;   /* off-diagonal, exact copy */
    xdd *e2;  /* e_i^2 in double-double */
    double tnorm;  /* ||T||_1 of the scaled matrix */
    double tnorm_in; /* ||T||_1 of the input */
    int sexp;      /* the data are the input times 2^-sexp */
    double pivmin; /* replacement for an exactly zero pivot */
    xdd gl, gu;    /* Gerschgorin interval */
} prob_t;

/* Preprocessing (Sec. 2): the entries are scaled by a power of two (exact
 * unless an entry falls below the normal range) so that ||T||_1 lies in
 * [1/2, 1); eigenvalues are scaled back on output, shifts and eigenvalues
 * passed in are scaled on input, and eigenvectors do not change.  Without it
 * the squares of very small or very large entries leave the exponent range. */
static void prob_init(prob_t *p, int n, const double *d_in, const double *e_in)
{
    p->n = n;
    p->d = (xdd *)malloc(sizeof(xdd) * (size_t)(n > 0 ? n : 1));
    p->e = (xdd *)malloc(sizeof(xdd) * (size_t)(n > 1 ? n - 1 : 1));
    p->e2 = (xdd *)malloc(sizeof(xdd) * (size_t)(n > 1 ? n - 1 : 1));
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *e = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
    double tn_in = 0.0;
    for (int i = 0; i < n; ++i) {
        double row = fabs(d_in[i]) + ((i > 0) ? fabs(e_in[i - 1]) : 0.0) +
                     ((i + 1 < n && ORACLE_MUTANT != 7) ? fabs(e_in[i]) : 0.0); /* mutant 7 */
        if (row > tn_in)
            tn_in = row;
    }
    p->tnorm_in = tn_in;
    p->sexp = 0;
    if (tn_in > 0.0 && isfinite(tn_in))
        (void)frexp(tn_in, &p->sexp);
    for (int i = 0; i < n; ++i)
        d[i] = ldexp(d_in[i], -p->sexp);
    for (int i = 0; i + 1 < n; ++i)
        e[i] = ldexp(e_in[i], -p->sexp);
    double tn = 0.0, emax2 = 0.0;
    double glo = 0.0, ghi = 0.0;
    for (int i = 0; i < n; ++i) {
        p->d[i] = from_d(d[i]);
        double left = (i > 0) ? fabs(e[i - 1]) : 0.0;
        double right = (i + 1 < n) ? fabs(e[i]) : 0.0;
        double row = left + fabs(d[i]) + ((ORACLE_MUTANT == 7) ? 0.0 : right); /* mutant 7 */
        if (row > tn)
            tn = row;
        double lo = d[i] - (left + right), hi = d[i] + (left + right);
        if (i == 0 || lo < glo)
            glo = lo;
        if (i == 0 || hi > ghi)
            ghi = hi;
    }
    for (int i = 0; i + 1 < n; ++i) {
        p->e[i] = from_d(e[i]);
        p->e2[i] = two_prod(e[i], e[i]);
        if (e[i] * e[i] > emax2)
            emax2 = e[i] * e[i];
    }
    p->tnorm = tn;
    p->pivmin = ldexp(1.0, -1000) * (emax2 > 1.0 ? emax2 : 1.0);
    double widen = ldexp(1.0, -50) * (ghi - glo) + ldexp(1.0, -50) * tn + 1e-300;
    p->gl = from_d(glo - widen);
    p->gu = from_d(ghi + widen);
    free(d);
    free(e);
}

/* x * 2^k for a double-double (exact while it stays in range) */
static xdd x_ldexp(xdd a, int k)
{
    return mk(ldexp(a.hi, k), ldexp(a.lo, k));
}

static void prob_free(prob_t *p)
{
    free(p->d);
    free(p->e);
    free(p->e2);
}

/* number of eigenvalues of T strictly below sigma (number of negative pivots
 * of T - sigma I, Sylvester's law of inertia).  An exactly zero pivot is
 * replaced by +pivmin: every pivot decreases as sigma grows, so this is the
 * count at sigma - 0, and an eigenvalue equal to sigma (a zero last pivot) is
 * not counted.  A zero pivot before the last row gives the same count with
 * either sign. */
static int sturm_count(const prob_t *p, xdd sigma)
{
    int cnt = 0;
    xdd q = from_d(0.0);
    for (int j = 0; j < p->n; ++j) {
        xdd t = x_sub(p->d[j], sigma);
        if (j > 0)
            t = (ORACLE_MUTANT == 1) ? x_sub(t, x_div(p->e[j - 1], q)) /* mutant: e, not e^2 */
                                     : x_sub(t, x_div(p->e2[j - 1], q));
        if (t.hi == 0.0 && t.lo == 0.0)
            t = from_d((ORACLE_MUTANT == 5) ? -p->pivmin : p->pivmin); /* mutant 5: sigma + 0 */
        if (t.hi < 0.0)
            ++cnt;
        q = t;
    }
    return cnt;
}

/* i-th smallest eigenvalue (1-based) by bisection to absolute width
 * 2^-96 ||T||_1, or until the midpoint no longer moves */
static xdd bisect_eig(const prob_t *p, int i)
{
    xdd lo = p->gl, hi = p->gu;
    double tol = ldexp(p->tnorm, -96);
    for (int it = 0; it < 400; ++it) {
        xdd w = x_sub(hi, lo);
        if (w.hi <= tol)
            break;
        xdd mid = x_mul_d(x_add(lo, hi), 0.5);
        if (x_eq(mid, lo) || x_eq(mid, hi))
            break;
        if (sturm_count(p, mid) >= i)
            hi = mid;
        else
            lo = mid;
    }
    return x_mul_d(x_add(lo, hi), 0.5);
}

/* ------------------------------------------------------------------------ */
/* inverse iteration                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    xdd *u0, *u1, *u2; /* U: diagonal, first and second super-diagonal */
    xdd *l;            /* multipliers */
    char *swp;         /* row interchange at step j */
} lu_t;

/* Gaussian elimination with partial pivoting of T - lambda I (tridiagonal).
 * A pivot that is exactly zero is replaced by a tiny multiple of ||T||_1. */
static void lu_factor(const prob_t *p, xdd lambda, lu_t *f)
{
    int n = p->n;
    f->n = n;
    /* working rows: current row has (a, b, c) in columns j, j+1, j+2 */
    xdd a = x_sub(p->d[0], lambda);
    xdd b = (n > 1) ? p->e[0] : from_d(0.0);
    xdd c = from_d(0.0);
    double tiny = ldexp(p->tnorm > 0 ? p->tnorm : 1.0, -104);
    for (int j = 0; j < n - 1; ++j) {
        /* next row: (e_j, d_{j+1} - lambda, e_{j+1}) in columns j, j+1, j+2 */
        xdd na = p->e[j];
        xdd nb = x_sub(p->d[j + 1], lambda);
        xdd nc = (j + 2 < n) ? p->e[j + 1] : from_d(0.0);
        if (x_lt(x_abs(a), x_abs(na))) {
            /* interchange: pivot row is the next row */
            f->swp[j] = 1;
            xdd m = x_div(a, na);
            f->u0[j] = na;
            f->u1[j] = nb;
            f->u2[j] = nc;
            f->l[j] = m;
            /* new current row = old current - m * pivot row, columns j+1, j+2 */
            xdd ra = x_sub(b, x_mul(m, nb));
            xdd rb = x_sub(c, x_mul(m, nc));
            a = ra;
            b = rb;
            c = from_d(0.0);
        } else {
            f->swp[j] = 0;
            if (a.hi == 0.0 && a.lo == 0.0 && ORACLE_MUTANT != 6) /* mutant 6: no guard */
                a = from_d(tiny);
            xdd m = x_div(na, a);
            f->u0[j] = a;
            f->u1[j] = b;
            f->u2[j] = c;
            f->l[j] = m;
            xdd ra = (ORACLE_MUTANT == 2) ? x_add(nb, x_mul(m, b)) /* mutant: sign */
                                          : x_sub(nb, x_mul(m, b));
            xdd rb = x_sub(nc, x_mul(m, c));
            a = ra;
            b = rb;
            c = from_d(0.0);
        }
    }
    if (a.hi == 0.0 && a.lo == 0.0 && ORACLE_MUTANT != 6)
        a = from_d(tiny);
    f->u0[n - 1] = a;
    f->u1[n - 1] = from_d(0.0);
    f->u2[n - 1] = from_d(0.0);
}

/* solve (T - lambda I) x = y in place using the factorisation */
static void lu_solve(const lu_t *f, xdd *x)
{
    int n = f->n;
    for (int j = 0; j < n - 1; ++j) {
        if (f->swp[j]) {
            xdd t = x[j];
            x[j] = x[j + 1];
            x[j + 1] = x_sub(t, x_mul(f->l[j], x[j]));
        } else {
            x[j + 1] = x_sub(x[j + 1], x_mul(f->l[j], x[j]));
        }
    }
    for (int j = n - 1; j >= 0; --j) {
        xdd s = x[j];
        if (j + 1 < n)
            s = x_sub(s, x_mul(f->u1[j], x[j + 1]));
        if (j + 2 < n)
            s = x_sub(s, x_mul(f->u2[j], x[j + 2]));
        x[j] = x_div(s, f->u0[j]);
    }
}

static xdd dot(int n, const xdd *a, const xdd *b)
{
    xdd s = from_d(0.0);
    for (int j = 0; j < n; ++j)
        s = x_add(s, x_mul(a[j], b[j]));
    return s;
}

static void normalise(int n, xdd *x)
{
    xdd nrm = x_sqrt(dot(n, x, x));
    if (nrm.hi == 0.0)
        return;
    for (int j = 0; j < n; ++j)
        x[j] = x_div(x[j], nrm);
}

/* splitmix64: seeded start vector entries in (-1, 1) */
static double start_entry(uint64_t seed, int idx, int j)
{
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + (uint64_t)idx * 0xD1B54A32D192ED03ull +
                 (uint64_t)j * 0x8CB92BA72F3D8DD7ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return ((double)(z >> 11) * ldexp(1.0, -53)) * 2.0 - 1.0;
}

/* ------------------------------------------------------------------------ */
/* public entry points                                                      */
/* ------------------------------------------------------------------------ */

/* Eigenvalues il..iu (1-based, inclusive) of T in double-double.
 * w_hi/w_lo receive iu-il+1 values.  nthreads <= 0 means all available. */
int oracle_eigvals(int n, const double *d, const double *e, int il, int iu,
                   double *w_hi, double *w_lo, int nthreads)
{
    if (n < 0 || il < 1 || iu > n || il > iu + 1)
        return -1;
    if (n == 0 || il > iu)
        return 0;
    prob_t p;
    prob_init(&p, n, d, e);
    int m = iu - il + 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads > 0 ? nthreads : omp_threads())
    for (int k = 0; k < m; ++k) {
        xdd lam = x_ldexp(bisect_eig(&p, il + k), p.sexp);
        w_hi[k] = lam.hi;
        w_lo[k] = lam.lo;
    }
    prob_free(&p);
    return 0;
}

/* Sturm count of T at sigma = s_hi + s_lo (double-double): number of
 * eigenvalues strictly below sigma. */
int oracle_count(int n, const double *d, const double *e, double s_hi, double s_lo)
{
    if (n <= 0)
        return 0;
    prob_t p;
    prob_init(&p, n, d, e);
    int c = sturm_count(&p, x_ldexp(mk(s_hi, s_lo), -p.sexp));
    prob_free(&p);
    return c;
}

/* Eigenvectors for the m eigenvalues w (double-double, ascending, as returned
 * by oracle_eigvals for il..iu).  z receives n*m values, column-major with
 * leading dimension n, rounded to double.  group_tol is the grouping distance
 * as a multiple of ||T||_1 (<= 0 selects 2^-60).  Returns 0 on success. */
int oracle_eigvecs(int n, const double *d, const double *e, int m, const double *w_hi,
                   const double *w_lo, double *z, unsigned long long seed, double group_tol,
                   int nthreads)
{
    if (n < 0 || m < 0 || m > n)
        return -1;
    if (n == 0 || m == 0)
        return 0;
    prob_t p;
    prob_init(&p, n, d, e);
    double gtol = (group_tol > 0 ? group_tol : ldexp(1.0, -60)) * p.tnorm;
    /* group boundaries: runs of consecutive eigenvalues closer than gtol */
    int *gstart = (int *)malloc(sizeof(int) * (size_t)(m + 1));
    int ng = 0;
    gstart[ng++] = 0;
    for (int k = 1; k < m; ++k) {
        xdd gap = x_ldexp(x_sub(mk(w_hi[k], w_lo[k]), mk(w_hi[k - 1], w_lo[k - 1])), -p.sexp);
        if (gap.hi > gtol)
            gstart[ng++] = k;
    }
    gstart[ng] = m;
    xdd *zz = (xdd *)malloc(sizeof(xdd) * (size_t)n * (size_t)m);
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : omp_threads())
    {
        lu_t f;
        f.u0 = (xdd *)malloc(sizeof(xdd) * (size_t)n);
        f.u1 = (xdd *)malloc(sizeof(xdd) * (size_t)n);
        f.u2 = (xdd *)malloc(sizeof(xdd) * (size_t)n);
        f.l = (xdd *)malloc(sizeof(xdd) * (size_t)n);
        f.swp = (char *)malloc((size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int g = 0; g < ng; ++g) {
            for (int k = gstart[g]; k < gstart[g + 1]; ++k) {
                xdd *x = zz + (size_t)k * (size_t)n;
                xdd lam = x_ldexp(mk(w_hi[k], w_lo[k]), -p.sexp);
                lu_factor(&p, lam, &f);
                for (int j = 0; j < n; ++j)
                    x[j] = from_d(start_entry(seed, k, j));
                normalise(n, x);
                int singleton = (gstart[g + 1] - gstart[g] == 1);
                int iters = singleton ? 4 : 6;
                for (int it = 0; it < iters; ++it) {
                    lu_solve(&f, x);
                    normalise(n, x);
                    for (int q = gstart[g]; q < k && ORACLE_MUTANT != 3; ++q) {
                        const xdd *y = zz + (size_t)q * (size_t)n;
                        xdd c = dot(n, y, x);
                        for (int j = 0; j < n; ++j)
                            x[j] = x_sub(x[j], x_mul(c, y[j]));
                    }
                    normalise(n, x);
                }
                /* sign: largest-magnitude entry positive */
                int jm = 0;
                for (int j = 1; j < n; ++j)
                    if (x_lt(x_abs(x[jm]), x_abs(x[j])))
                        jm = j;
                if (x[jm].hi < 0.0)
                    for (int j = 0; j < n; ++j)
                        x[j] = x_neg(x[j]);
            }
        }
        free(f.u0);
        free(f.u1);
        free(f.u2);
        free(f.l);
        free(f.swp);
    }
    for (size_t t = 0; t < (size_t)n * (size_t)m; ++t)
        z[t] = x_to_d(zz[t]);
    free(zz);
    free(gstart);
    prob_free(&p);
    return 0;
}

/* ||T||_1 as the oracle computes it (max absolute row sum) */
double oracle_tnorm(int n, const double *d, const double *e)
{
    if (n <= 0)
        return 0.0;
    prob_t p;
    prob_init(&p, n, d, e);
    double t = p.tnorm_in;
    prob_free(&p);
    return t;
}

/* exposed double-double primitives, for pinning them against exact rationals */
void oracle_dd_op(int op, double ahi, double alo, double bhi, double blo, double *rhi, double *rlo)
{
    xdd a = mk(ahi, alo), b = mk(bhi, blo), r;
    switch (op) {
    case 0: r = x_add(a, b); break;
    case 1: r = x_sub(a, b); break;
    case 2: r = x_mul(a, b); break;
    case 3: r = x_div(a, b); break;
    default: r = x_sqrt(a); break;
    }
    *rhi = r.hi;
    *rlo = r.lo;
}

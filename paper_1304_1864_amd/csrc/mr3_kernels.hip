// HIP kernels of the mixed-precision MRRR hot path (gfx950).
//
// Algorithm 1 of the paper (MRRR), with the mixed precision adjustments of its
// Section 3.2, mapped onto the GPU level by level:
//   k_prep      preprocessing: ||T||_1, power-of-two scaling, splitting,
//               per-block Gerschgorin bounds and requested index ranges
//   k_root      root representation M_root = T - mu I (definite, mu just
//               outside the spectrum) and its random relative perturbation
//               (Alg. 1, root step; Sec. 3.2 "Random perturbations")
//   k_pq        off-diagonal prefix/suffix products used by the eigenvector
//               recurrences (shared by every node of a tree)
//   k_bisect    multisection on Sturm counts of a binary64 copy of a
//               representation (Alg. 1, eigenvalue and refine steps;
//               Sec. 3.2 "Arithmetic used to approximate eigenvalues");
//               k_bisect_staged streams the rows of large nodes through LDS
//               or keeps those of small ones resident, k_slice and
//               k_slice_small share counts among all eigenvalues of a root
//   k_dqds      optional initial eigenvalues of whole spectra by the dqds
//               algorithm, one lane per root (Sec. 4.1), checked and refined
//               by the multisection afterwards
//   k_classify  singleton / cluster partition by reldist >= gaptol (Alg. 1,
//               classification step; Sec. 2 "Classification of the eigenvalues")
//   k_rqi       Rayleigh quotient iteration with twisted factorizations
//               (Alg. 1, singleton step; Sec. 2 "Rayleigh quotient iteration",
//               Sec. 3.2 stopping criterion)
//   k_zout      eigenvector normalisation, y -> x rounding, coalesced Z stores
//   k_child_*   cluster shifts M - tau I by the stationary qd transform in y
//               with an element-growth acceptance test (Alg. 1, shift step;
//               Sec. 2 "Shifting the spectrum", "Requirements on the
//               representations")
//
// Recurrences.  For a representation L D L^T (data d_i and lld_i = d_i l_i^2,
// off-diagonals e_i = d_i l_i shared by all nodes of a tree) and a shift tau,
// the stationary transform L D L^T - tau I = L+ D+ L+^T runs
//     s_1 = -tau,  d+_i = d_i + s_i,  s_{i+1} = lld_i s_i / d+_i - tau
// and the progressive one L D L^T - tau I = U Omega U^T runs
//     p_n = d_n - tau,  w_{i+1} = lld_i + p_{i+1},  p_i = d_i p_{i+1} / w_{i+1} - tau.
// Both are evaluated here in an equivalent division-free form: writing
// s_i = a_i / b_i gives  c_i = d_i b_i + a_i  (= d+_i b_i),
// a_{i+1} = lld_i a_i - tau c_i,  b_{i+1} = c_i;  writing p_i = alpha_i / beta_i
// gives  rho_{i+1} = lld_i beta_{i+1} + alpha_{i+1}  (= w_{i+1} beta_{i+1}),
// alpha_i = d_i alpha_{i+1} - tau rho_{i+1},  beta_i = rho_{i+1}.  Each sum is
// one rounding of the same operands as in the divided form, so the mixed
// relative stability of the qd transforms carries over; the pairs are rescaled
// by powers of two (exact) to stay in range.  sign(d+_i) = sign(c_i) sign(b_i)
// gives the Sturm count (Sylvester inertia) without a division.
// The twisted factorization at index r has gamma_r = s_r + p_r + tau, and the
// solution of N_r^T z = e_r is, up to scaling,
//     z_k = P_k b_k      (k <= r),   P_k = prod_{j<k} (-1/e_j)
//     z_k = Q_k beta_k   (k >= r),   Q_k = prod_{j>=k} (-1/e_j)
// which follows from z_{k+1} = -z_k d+_k / e_k and z_k = -z_{k+1} w_{k+1} / e_k.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd.hpp"
#include "mr3_types.hpp"

namespace mr3 {

#define MR3_BIG 1.0e300

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dexp(double x) { return __builtin_amdgcn_frexp_exp(x); }

// rows per LDS window of the staged sweeps = threads per workgroup
constexpr int STAGE_ROWS = 256;

__device__ __forceinline__ int sign_differs(double c, double b) {
    return (int)(((unsigned)__double2hiint(c) ^ (unsigned)__double2hiint(b)) >> 31);
}

// counter-based generator (splitmix64 finaliser) -> uniform in [-1, 1)
__device__ __forceinline__ double urand_pm1(unsigned long long seed, unsigned long long row,
                                            unsigned long long arr) {
    unsigned long long z = seed * 0x9E3779B97F4A7C15ull + row * 0xBF58476D1CE4E5B9ull +
                           (arr + 1ull) * 0x94D049BB133111EBull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 2.220446049250313e-16 - 1.0;  // 2^-52 * [0, 2^53) - 1
}

// Sturm count of the tridiagonal (Td, Te) rows [0, n) at x: number of
// eigenvalues below x (negative pivots of T - x I); used only in the
// preprocessing, not on the hot path.
__device__ int sturm_T(const double* __restrict__ Td, const double* __restrict__ Te, int64_t n,
                       double x) {
    const double pivmin = 1e-290;
    int cnt = 0;
    double q = 1.0;
    for (int64_t i = 0; i < n; ++i) {
        double off = (i > 0) ? Te[i - 1] : 0.0;
        double t = Td[i] - x;
        if (off != 0.0) t -= (off * off) / q;
        if (fabs(t) < pivmin) t = -pivmin;
        cnt += (t < 0.0);
        q = t;
    }
    return cnt;
}

// Sturm counts at P shifts in one pass over the rows: the row loads are shared
// and the P recurrences are independent chains that fill the FP64 pipeline.
template <int P>
__device__ __forceinline__ void negcount64_multi(const double* __restrict__ D,
                                                 const double* __restrict__ LL, int64_t n,
                                                 const double (&x)[P], int (&neg)[P]) {
    // rows per block: the next block's loads are in flight while a block is
    // processed, so fewer chains get longer blocks to cover memory latency
    constexpr int U = (P == 1) ? 16 : 8;
    double a[P], b[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        a[p] = -x[p];
        b[p] = 1.0;
        neg[p] = 0;
    }
    if (n <= 0) return;
    double dn[U], ln[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        dn[u] = D[u];
        ln[u] = LL[u];
    }
    int64_t i = 0;
    // full blocks: straight-line code, the next block's loads in flight
    for (; i + U <= n; i += U) {
        double dc[U], lc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dc[u] = dn[u];
            lc[u] = ln[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dn[u] = D[i + U + u];
            ln[u] = LL[i + U + u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const double c = __fma_rn(dc[u], b[p], a[p]);
                neg[p] += sign_differs(c, b[p]);
                a[p] = __fma_rn(-x[p], c, lc[u] * a[p]);
                b[p] = c;
            }
            if ((u & 3) == 3) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const int em = max(dexp(a[p]), dexp(b[p]));
                    a[p] = __builtin_ldexp(a[p], -em);
                    b[p] = __builtin_ldexp(b[p], -em);
                }
            }
        }
    }
    // tail (fewer than U rows), already loaded in dn/ln
    for (int u = 0; u < U && i + u < n; ++u) {
        const double du = dn[0], lu = ln[0];
#pragma unroll
        for (int v = 0; v + 1 < U; ++v) {
            dn[v] = dn[v + 1];
            ln[v] = ln[v + 1];
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double c = __fma_rn(du, b[p], a[p]);
            neg[p] += sign_differs(c, b[p]);
            a[p] = __fma_rn(-x[p], c, lu * a[p]);
            b[p] = c;
        }
    }
}

// Sturm count of the binary64 representation (d, lld) at one shift x
__device__ __forceinline__ int negcount64(const double* __restrict__ D,
                                          const double* __restrict__ LL, int64_t n, double x) {
    const double xs[1] = {x};
    int c[1];
    negcount64_multi<1>(D, LL, n, xs, c);
    return c[0];
}

// Sturm count of the scaled tridiagonal (Td, Te) rows [0, n) at x, division
// free: the leading minors p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2} change
// sign once per negative pivot of T - x I.  Same double buffering as
// negcount64 (guard rows behind the arrays).
__device__ __forceinline__ int negcount_T(const double* __restrict__ Td,
                                          const double* __restrict__ Te, int64_t n, double x) {
    constexpr int U = 8;
    if (n <= 0) return 0;
    double pm = 0.0, p = 1.0;  // p_{i-2}, p_{i-1} (p_0 = 1, p_{-1} unused)
    int neg = 0;
    double dn[U], en[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        dn[u] = Td[u];
        en[u] = (u > 0) ? Te[u - 1] : 0.0;
    }
    for (int64_t i = 0; i < n; i += U) {
        double dc[U], ec[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dc[u] = dn[u];
            ec[u] = en[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dn[u] = Td[i + U + u];
            en[u] = Te[i + U + u - 1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i + u < n) {
                const double pn = __fma_rn(dc[u] - x, p, -(ec[u] * ec[u]) * pm);
                neg += sign_differs(pn, p);
                pm = p;
                p = pn;
                if ((u & 3) == 3) {
                    const int em = max(dexp(p), dexp(pm));
                    p = __builtin_ldexp(p, -em);
                    pm = __builtin_ldexp(pm, -em);
                }
            }
        }
    }
    return neg;
}

// lld_i = e_i^2 / d_i of a node in y: the stored array, or, when nodes keep
// only d (the e-representation, Sec. 3.2 "Choice of representations": the
// off-diagonals e are the same for every node of a block and stored once),
// formed from the block's e and the node's d by the formula that would have
// stored it (so both ways give the same bits).  Rows outside [0, n-1) give 0.
template <class Y>
__device__ __forceinline__ Y lld_at(const Y* __restrict__ LL, const Y* __restrict__ E,
                                    const Y* __restrict__ D, int64_t i, int64_t n) {
    if (LL) return LL[i];
    return (i >= 0 && i + 1 < n) ? div(mul(E[i], E[i]), D[i]) : y_from(0.0, Y());
}

// the same count in working precision y (DL: lld from E and D)
template <class Y, bool DL>
__device__ int negcount_y(const Y* __restrict__ D, const Y* __restrict__ LL,
                          const Y* __restrict__ E, int64_t n, Y x) {
    Y a = neg(x), b = y_from(1.0, Y());
    int neg_ = 0;
    for (int64_t i = 0; i < n; ++i) {
        Y c = mul_add(D[i], b, a);
        neg_ += sign_differs(hi_of(c), hi_of(b));
        a = mul_sub(DL ? lld_at<Y>(nullptr, E, D, i, n) : LL[i], a, x, c);
        b = c;
        if ((i & 3) == 3) {
            const int em = max(y_exp(a), y_exp(b));
            a = y_ldexp(a, -em);
            b = y_ldexp(b, -em);
        }
    }
    return neg_;
}

__device__ __forceinline__ double block_reduce_max(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// a1: preprocessing (one workgroup of 256 per problem)
// ---------------------------------------------------------------------------
// Index-range resolution for a split problem: find x with count(x) <= c on
// the split matrix, as close as the arithmetic allows to the eigenvalue c+1,
// and the per-block counts there; eigenvalues that tie across blocks inside
// the final bracket are handed to blocks in block order.
__device__ void index_boundary(const double* Td, const double* Te, int64_t n, double glo,
                               double ghi, int64_t c, int nb, BlockInfo* bi, int which,
                               double* sh_x, int* sh_c) {
    const int t = threadIdx.x;
    __shared__ double s_lo, s_hi;
    __shared__ int s_done;
    if (t == 0) {
        s_lo = glo;
        s_hi = ghi;
        s_done = (c <= 0) ? 1 : 0;
    }
    __syncthreads();
    for (int round = 0; round < 12 && !s_done; ++round) {
        const double lo = s_lo, hi = s_hi;
        const double x = lo + (hi - lo) * ((double)(t + 1) / 256.0);
        sh_x[t] = x;
        sh_c[t] = (t < 255) ? sturm_T(Td, Te, n, x) : (int)n;
        __syncthreads();
        if (t == 0) {
            int f = 255;  // first point with count > c
            for (int q = 0; q < 255; ++q)
                if (sh_c[q] > c) { f = q; break; }
            const double nlo = (f > 0) ? sh_x[f - 1] : lo;
            const double nhi = (f < 255) ? sh_x[f] : hi;
            if (f > 0 && sh_c[f - 1] == c) s_done = 1;
            if (nlo == s_lo && nhi == s_hi) s_done = 1;
            s_lo = nlo;
            s_hi = nhi;
        }
        __syncthreads();
    }
    const double xlo = s_lo, xhi = s_hi;
    // per-block counts at both ends of the final bracket
    for (int b = t; b < nb; b += blockDim.x) {
        const int64_t s = bi[b].start;
        const int64_t e_ = (b + 1 < nb) ? bi[b + 1].start : n;
        int clo = (c <= 0) ? 0 : sturm_T(Td + s, Te + s, e_ - s, xlo);
        int chi = (c <= 0) ? 0 : sturm_T(Td + s, Te + s, e_ - s, xhi);
        if (which == 0) {
            bi[b].il = clo;
            bi[b].gl = (double)chi;  // temporary: count at the upper end
        } else {
            bi[b].iu = clo;
            bi[b].gu = (double)chi;
        }
    }
    __syncthreads();
    if (t == 0) {
        int64_t total = 0;
        for (int b = 0; b < nb; ++b) total += (which == 0) ? bi[b].il : bi[b].iu;
        int64_t deficit = c - total;
        for (int b = 0; b < nb && deficit > 0; ++b) {
            const int64_t room = (int64_t)((which == 0) ? bi[b].gl : bi[b].gu) -
                                 ((which == 0) ? bi[b].il : bi[b].iu);
            const int64_t take = room < deficit ? room : deficit;
            if (which == 0) bi[b].il += take; else bi[b].iu += take;
            deficit -= take;
        }
    }
    __syncthreads();
}

template <class X>
__global__ void __launch_bounds__(256)
k_prep(const ProbDesc* __restrict__ probs, double eps_x, double* __restrict__ Td, double* __restrict__ Te, ProbInfo* __restrict__ info,
       BlockInfo* __restrict__ binfo) {
    __shared__ double sh[256];
    __shared__ int shi[256];
    const int p = blockIdx.x;
    const int t = threadIdx.x;
    const ProbDesc pd = probs[p];
    const int64_t n = pd.n;
    const X* d = reinterpret_cast<const X*>(pd.din);
    const X* e = reinterpret_cast<const X*>(pd.ein);
    double* td = Td + pd.row0;
    double* te = Te + pd.row0;
    BlockInfo* bi = binfo + pd.row0;
    if (n == 0) {
        if (t == 0) { info[p].nblocks = 0; info[p].err = 0; info[p].sexp = 0; info[p].tnorm = 0; }
        return;
    }
    // ||T||_1 and finiteness
    double rmax = 0.0;
    int bad = 0;
    for (int64_t i = t; i < n; i += blockDim.x) {
        const double di = (double)d[i];
        const double el = (i > 0) ? fabs((double)e[i - 1]) : 0.0;
        const double er = (i + 1 < n) ? fabs((double)e[i]) : 0.0;
        if (!isfinite(di) || !isfinite(el) || !isfinite(er)) bad = 1;
        rmax = fmax(rmax, el + fabs(di) + er);
    }
    shi[t] = bad;
    const double tnorm = block_reduce_max(rmax, sh);
    int anybad = 0;
    for (int q = 0; q < 256; ++q) anybad |= shi[q];
    if (anybad) {
        if (t == 0) { info[p].err = 1; info[p].nblocks = 0; }
        return;
    }
    const int sexp = (tnorm > 0.0) ? -dexp(tnorm) : 0;
    const double tn = __builtin_ldexp(tnorm, sexp);
    const double thresh = eps_x * tn;
    for (int64_t i = t; i < n; i += blockDim.x) {
        td[i] = __builtin_ldexp((double)d[i], sexp);
        double ev = 0.0;
        if (i + 1 < n) {
            ev = __builtin_ldexp((double)e[i], sexp);
            if (fabs(ev) <= thresh) ev = 0.0;  // split (Sec. 3.2 "Preprocessing")
        }
        te[i] = ev;
    }
    __syncthreads();
    // block starts: row i starts a block if i == 0 or e_{i-1} was set to zero
    const int64_t chunk = (n + blockDim.x - 1) / blockDim.x;
    const int64_t c0 = t * chunk, c1 = min(n, c0 + chunk);
    int cnt = 0;
    for (int64_t i = c0; i < c1; ++i) cnt += (i == 0 || te[i - 1] == 0.0);
    shi[t] = cnt;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int q = 0; q < 256; ++q) { int v = shi[q]; shi[q] = run; run += v; }
        info[p].nblocks = run;
        info[p].sexp = sexp;
        info[p].tnorm = tn;
        info[p].err = 0;
    }
    __syncthreads();
    int pos = shi[t];
    for (int64_t i = c0; i < c1; ++i)
        if (i == 0 || te[i - 1] == 0.0) bi[pos++].start = i;
    __syncthreads();
    const int nb = info[p].nblocks;
    if (nb == 1) {
        // one block: Gerschgorin bounds by a workgroup reduction, the two
        // value-range counts on two threads
        double gl = MR3_BIG, gu = -MR3_BIG;
        for (int64_t i = t; i < n; i += blockDim.x) {
            const double off = ((i > 0) ? fabs(te[i - 1]) : 0.0) + ((i + 1 < n) ? fabs(te[i]) : 0.0);
            gl = fmin(gl, td[i] - off);
            gu = fmax(gu, td[i] + off);
        }
        gl = -block_reduce_max(-gl, sh);
        gu = block_reduce_max(gu, sh);
        if (pd.range == RANGE_VALUE && t < 2) {
            const double v = __builtin_ldexp(t == 0 ? pd.vl : pd.vu, sexp);
            shi[t] = negcount_T(td, te, n, v);
        }
        __syncthreads();
        if (t == 0) {
            bi[0].n = n;
            if (pd.range == RANGE_VALUE) {
                bi[0].il = shi[0] + 1;
                bi[0].iu = shi[1];
            } else if (pd.range == RANGE_INDEX) {
                bi[0].il = pd.il;
                bi[0].iu = pd.iu;
            } else {
                bi[0].il = 1;
                bi[0].iu = n;
            }
            bi[0].gl = gl;
            bi[0].gu = gu;
        }
        return;
    }
    for (int b = t; b < nb; b += blockDim.x) {
        const int64_t s = bi[b].start;
        const int64_t en = (b + 1 < nb) ? bi[b + 1].start : n;
        double gl = MR3_BIG, gu = -MR3_BIG;
        for (int64_t i = s; i < en; ++i) {
            const double off = ((i > s) ? fabs(te[i - 1]) : 0.0) + ((i + 1 < en) ? fabs(te[i]) : 0.0);
            gl = fmin(gl, td[i] - off);
            gu = fmax(gu, td[i] + off);
        }
        bi[b].n = en - s;
        if (pd.range == RANGE_VALUE) {
            const double vl = __builtin_ldexp(pd.vl, sexp), vu = __builtin_ldexp(pd.vu, sexp);
            bi[b].il = sturm_T(td + s, te + s, en - s, vl) + 1;
            bi[b].iu = sturm_T(td + s, te + s, en - s, vu);
        } else if (pd.range == RANGE_INDEX && nb == 1) {
            bi[b].il = pd.il;
            bi[b].iu = pd.iu;
        } else {
            bi[b].il = 1;
            bi[b].iu = en - s;
        }
        bi[b].gl = gl;
        bi[b].gu = gu;
    }
    __syncthreads();
    if (pd.range == RANGE_INDEX && nb > 1) {
        double glo = MR3_BIG, ghi = -MR3_BIG;
        for (int b = 0; b < nb; ++b) { glo = fmin(glo, bi[b].gl); ghi = fmax(ghi, bi[b].gu); }
        // keep the Gerschgorin bounds; the boundary search uses il/iu and
        // gl/gu of the block records as scratch, so save them first
        __shared__ double s_gl[1], s_gu[1];
        (void)s_gl; (void)s_gu;
        const double span = fmax(ghi - glo, 1e-300);
        glo -= 1e-3 * span;
        ghi += 1e-3 * span;
        // stash Gerschgorin bounds in Te-adjacent scratch: recompute afterwards
        index_boundary(td, te, n, glo, ghi, pd.il - 1, nb, bi, 0, sh, shi);
        index_boundary(td, te, n, glo, ghi, pd.iu, nb, bi, 1, sh, shi);
        for (int b = t; b < nb; b += blockDim.x) {
            const int64_t s = bi[b].start;
            const int64_t en = s + bi[b].n;
            bi[b].il = bi[b].il + 1;  // first requested local index
            double gl = MR3_BIG, gu = -MR3_BIG;
            for (int64_t i = s; i < en; ++i) {
                const double off = ((i > s) ? fabs(te[i - 1]) : 0.0) + ((i + 1 < en) ? fabs(te[i]) : 0.0);
                gl = fmin(gl, td[i] - off);
                gu = fmax(gu, td[i] + off);
            }
            bi[b].gl = gl;
            bi[b].gu = gu;
        }
    }
}

// ---------------------------------------------------------------------------
// a2: root representation (one workgroup of 256 per block)
// ---------------------------------------------------------------------------
template <class Y>
__global__ void __launch_bounds__(256)
k_root(const Block* __restrict__ blocks, const double* __restrict__ Td,
       const double* __restrict__ Te, Params prm, Y* __restrict__ rep_d, Y* __restrict__ rep_lld,
       Y* __restrict__ rep_e, double* __restrict__ d64, double* __restrict__ lld64,
       Node* __restrict__ nodes, Slot* __restrict__ slots, int* __restrict__ status) {
    __shared__ double sx[256];
    __shared__ int sc[256];
    __shared__ double2 wT[2][STAGE_ROWS];
    __shared__ double s_lo, s_hi, s_mu;
    __shared__ int s_ok, s_right;
    const int bidx = blockIdx.x;
    const int t = threadIdx.x;
    const Block blk = blocks[bidx];
    const int64_t n = blk.n;
    if (n == 0) return;
    const double* td = Td + blk.row0;
    const double* te = Te + blk.row0;
    const double gl = blk.gl, gu = blk.gu;
    const double spd = fmax(gu - gl, 1e-300);
    // The block's rows (d_i, e_{i-1}^2) stream through an LDS window shared by
    // the workgroup, so the sequential loops below read LDS, not memory.
    // Every thread calls these helpers (they synchronise the workgroup).
    auto load_row = [&](int64_t i) -> double2 {
        if (i >= n) return make_double2(0.0, 0.0);
        const double ei = (i > 0) ? te[i - 1] : 0.0;
        return make_double2(td[i], ei * ei);
    };
    // Sturm count of T - x I (division free: leading minors p_i change sign
    // once per negative pivot), for threads with on == true
    auto tcount = [&](double x, bool on) -> int {
        double pm = 0.0, p = 1.0;
        int neg = 0;
        wT[0][t] = load_row(t);
        __syncthreads();
        for (int64_t c0 = 0; c0 < n; c0 += STAGE_ROWS) {
            const int cur = (int)((c0 / STAGE_ROWS) & 1);
            const double2 nx = load_row(c0 + STAGE_ROWS + t);
            const int cnt = (int)min<int64_t>(STAGE_ROWS, n - c0);
            if (on) {
                auto row = [&](const double2& r, int i) {
                    const double pn = __fma_rn(r.x - x, p, -r.y * pm);
                    neg += sign_differs(pn, p);
                    pm = p;
                    p = pn;
                    if ((i & 3) == 3) {
                        const int em = max(dexp(p), dexp(pm));
                        p = __builtin_ldexp(p, -em);
                        pm = __builtin_ldexp(pm, -em);
                    }
                };
                int i = 0;
                for (; i + 8 <= cnt; i += 8) {
                    double2 r[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) r[u] = wT[cur][i + u];
#pragma unroll
                    for (int u = 0; u < 8; ++u) row(r[u], i + u);
                }
                for (; i < cnt; ++i) row(wT[cur][i], i);
            }
            wT[cur ^ 1][t] = nx;
            __syncthreads();
        }
        return neg;
    };
    // round 0: 254 points over the whole interval bracket both extreme
    // eigenvalues, and two threads count at the quarter points, which choose
    // the end: all eigenvalues -> the more populated end; a subset -> the end
    // nearer to the requested indices
    {
        const double lo = gl - 1e-3 * spd, hi = gu + 1e-3 * spd;
        double x;
        if (t < 254) x = lo + (hi - lo) * ((double)(t + 1) / 255.0);
        else x = (t == 254) ? gl + 0.25 * spd : gu - 0.25 * spd;
        sx[t] = x;
        sc[t] = tcount(x, true);
        __syncthreads();
        if (t == 0) {
            int right;
            if (blk.il == 1 && blk.iu == n) right = ((int64_t)n - sc[255] > sc[254]) ? 1 : 0;
            else right = (blk.il + blk.iu > n + 1) ? 1 : 0;
            s_right = right;
            const int64_t target = right ? n - 1 : 0;
            int f = 254;
            for (int q = 0; q < 254; ++q)
                if (sc[q] > target) { f = q; break; }
            s_lo = (f > 0) ? sx[f - 1] : lo;
            s_hi = (f < 254) ? sx[f] : hi;
        }
        __syncthreads();
    }
    const int right = s_right;
    // one more round of 255-point multisection on the chosen end brackets the
    // extreme eigenvalue to spdiam / 2^16, well inside the distance that mu
    // keeps from it (below)
    const int64_t target = right ? n - 1 : 0;  // count threshold
    for (int round = 0; round < 1; ++round) {
        const double lo = s_lo, hi = s_hi;
        const double x = lo + (hi - lo) * ((double)(t + 1) / 256.0);
        sx[t] = x;
        const int c = tcount(x, t < 255);
        sc[t] = (t < 255) ? c : (int)n;
        __syncthreads();
        if (t == 0) {
            int f = 255;
            for (int q = 0; q < 255; ++q)
                if (sc[q] > target) { f = q; break; }
            s_lo = (f > 0) ? sx[f - 1] : lo;
            s_hi = (f < 255) ? sx[f] : hi;
        }
        __syncthreads();
    }
    // shift and factor T - mu I = L D L^T in binary64 (continuant form:
    // q_i = (a_i - mu) q_{i-1} - e_{i-1}^2 q_{i-2},  d_i = q_i / q_{i-1}) by
    // thread 0, rows from the LDS window
    // mu stays at least 10^-3 spdiam outside the spectrum: the eigenvalues of
    // M then all have |lambda| >= 10^-3 spdiam, so bisection to a relative
    // width costs about as many passes at that end as anywhere else, and the
    // relative gaps there only lose what a 10^-3 spdiam move of the origin
    // takes
    double delta = fmax(fmax(2.0 * (s_hi - s_lo), 8.0 * (double)n * 1.1102230246251565e-16),
                        prm.root_gap * spd);
    // The serial lane stores each continuant q_i as computed and, after rows
    // 4k+3, the exponent em by which q and q_{i-1} were then scaled down;
    // the pivots d_i = q_i / q_{i-1} (times 2^em across a rescaling, exact)
    // are formed afterwards by all threads, so no division is on the serial
    // lane's instruction stream.  q_i goes to d64, em to lld64 (both rewritten
    // below).
    double* qst = d64 + blk.row0;
    double* est = lld64 + blk.row0;
    for (int attempt = 0; attempt < 40; ++attempt) {
        const double mu = right ? s_hi + delta : s_lo - delta;
        double qm = 1.0, q = 1.0;
        wT[0][t] = load_row(t);
        __syncthreads();
        for (int64_t c0 = 0; c0 < n; c0 += STAGE_ROWS) {
            const int cur = (int)((c0 / STAGE_ROWS) & 1);
            const double2 nx = load_row(c0 + STAGE_ROWS + t);
            const int cnt = (int)min<int64_t>(STAGE_ROWS, n - c0);
            if (t == 0) {
                auto row = [&](const double2& r, int i) {
                    const double qn = __fma_rn(r.x - mu, q, -r.y * qm);
                    qst[c0 + i] = qn;
                    qm = q;
                    q = qn;
                    int em = 0;
                    if ((i & 3) == 3) {
                        em = max(dexp(q), dexp(qm));
                        q = __builtin_ldexp(q, -em);
                        qm = __builtin_ldexp(qm, -em);
                    }
                    est[c0 + i] = (double)em;
                };
                int i = 0;
                for (; i + 8 <= cnt; i += 8) {
                    double2 r[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) r[u] = wT[cur][i + u];
#pragma unroll
                    for (int u = 0; u < 8; ++u) row(r[u], i + u);
                }
                for (; i < cnt; ++i) row(wT[cur][i], i);
            }
            wT[cur ^ 1][t] = nx;
            __syncthreads();
        }
        // pivots, and the definiteness check: every d_i of one sign
        int bad = 0;
        for (int64_t i = t; i < n; i += blockDim.x) {
            const double di = (i == 0) ? qst[0] : __builtin_ldexp(qst[i] / qst[i - 1], (int)est[i - 1]);
            bad |= right ? !(di < 0.0) : !(di > 0.0);
            rep_d[blk.row0 + i] = y_from(di, Y());  // staged (rewritten below)
        }
        const int anybad = __syncthreads_or(bad);
        for (int64_t i = t; i < n; i += blockDim.x) d64[blk.row0 + i] = hi_of(rep_d[blk.row0 + i]);
        if (t == 0) {
            s_mu = mu;
            s_ok = !anybad;
        }
        __syncthreads();
        if (s_ok) break;
        delta *= 4.0;
        __syncthreads();
    }
    if (!s_ok) {
        if (t == 0) atomicOr(status, 1);
        return;
    }
    const double mu = s_mu;
    // random relative perturbation of the data in y (Alg. 1, root step), keyed by
    // the row index within the problem so that results do not depend on how
    // problems are batched
    const Y one = y_from(1.0, Y());
    for (int64_t i = t; i < n; i += blockDim.x) {
        const unsigned long long row = (unsigned long long)(blk.start + i);
        const unsigned long long key = prm.seed;
        const double xi_d = prm.xi * urand_pm1(key, row, 0);
        Y dt = mul(y_from(d64[blk.row0 + i], Y()), add_acc(one, y_from(xi_d, Y())));
        // a block of one row has its entry as eigenvalue: its pivot is formed
        // in y from the entry (exact on the double-double path) and not
        // perturbed, since there is no cluster to break up
        if (n == 1) dt = sub(y_from(td[0], Y()), y_from(mu, Y()));
        rep_d[blk.row0 + i] = dt;
    }
    __syncthreads();
    for (int64_t i = t; i < n; i += blockDim.x) {
        const unsigned long long row = (unsigned long long)(blk.start + i);
        const unsigned long long key = prm.seed;
        const Y dt = rep_d[blk.row0 + i];
        Y ll = y_from(0.0, Y());
        Y et = y_from(0.0, Y());
        if (i + 1 < n) {
            const double xi_e = prm.xi * urand_pm1(key, row, 1);
            et = mul(y_from(te[i], Y()), add_acc(one, y_from(xi_e, Y())));
            ll = div(mul(et, et), dt);
        }
        rep_e[blk.row0 + i] = et;
        if (rep_lld) rep_lld[blk.row0 + i] = ll;
        d64[blk.row0 + i] = to_double(dt);
        lld64[blk.row0 + i] = to_double(ll);
    }
    // root node and initial intervals of the block's slots
    const double slack = 16.0 * prm.xi + 64.0 * 1.1102230246251565e-16;
    double ilo, ihi;
    if (right) {
        ilo = (gl - mu) * (1.0 + slack) - 1e-300;
        ihi = 0.0;
    } else {
        ilo = 0.0;
        ihi = (gu - mu) * (1.0 + slack) + 1e-300;
    }
    if (t == 0) {
        Node nd;
        nd.block = bidx;
        nd.depth = 0;
        nd.rep = blk.row0;
        nd.first = blk.slot0;
        nd.last = blk.slot0 + blk.nslot - 1;
        nd.sigma_hi = mu;
        nd.sigma_lo = 0.0;
        nd.spdiam = spd;
        nodes[bidx] = nd;
    }
    for (int64_t s = blk.slot0 + t; s < blk.slot0 + blk.nslot; s += blockDim.x) {
        slots[s].node = bidx;
        slots[s].lo = ilo;
        slots[s].hi = ihi;
    }
}

// ---------------------------------------------------------------------------
// eigenvector products P_k = prod_{j<k} (-1/e_j), Q_k = prod_{j>=k, j<n-1} (-1/e_j)
// kept as (y mantissa, binary exponent); one workgroup of 256 per block
// ---------------------------------------------------------------------------
template <class Y>
__device__ __forceinline__ void normalise(Y& m, int& e) {
    const int k = y_exp(m);
    m = y_ldexp(m, -k);
    e += k;
}

template <class Y>
__global__ void __launch_bounds__(256)
k_pq(const Block* __restrict__ blocks, const Y* __restrict__ rep_e, Y* __restrict__ P,
     int* __restrict__ Pe, Y* __restrict__ Q, int* __restrict__ Qe, double* __restrict__ P64,
     double* __restrict__ Q64) {
    __shared__ Y sm[256];
    __shared__ int se[256];
    const Block blk = blocks[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t n = blk.n;
    if (n == 0) return;
    const Y* e = rep_e + blk.row0;
    const int64_t chunk = (n + blockDim.x - 1) / blockDim.x;
    const int64_t c0 = min(n, (int64_t)t * chunk), c1 = min(n, c0 + chunk);
    const Y one = y_from(1.0, Y());
    // prefix products
    Y m = one;
    int ex = 0;
    for (int64_t j = c0; j < c1; ++j)
        if (j + 1 < n) { m = mul(m, neg(div(one, e[j]))); normalise(m, ex); }
    sm[t] = m;
    se[t] = ex;
    __syncthreads();
    if (t == 0) {
        Y run = one;
        int re = 0;
        for (int q = 0; q < (int)blockDim.x; ++q) {
            Y v = sm[q];
            int ve = se[q];
            sm[q] = run;
            se[q] = re;
            run = mul(run, v);
            re += ve;
            normalise(run, re);
        }
    }
    __syncthreads();
    m = sm[t];
    ex = se[t];
    for (int64_t j = c0; j < c1; ++j) {
        P[blk.row0 + j] = m;
        Pe[blk.row0 + j] = ex;
        if (P64) P64[blk.row0 + j] = hi_of(m);  // binary64 mantissa, same exponent
        if (j + 1 < n) { m = mul(m, neg(div(one, e[j]))); normalise(m, ex); }
    }
    __syncthreads();
    // suffix products
    m = one;
    ex = 0;
    for (int64_t j = c1 - 1; j >= c0; --j)
        if (j + 1 < n) { m = mul(m, neg(div(one, e[j]))); normalise(m, ex); }
    sm[t] = m;
    se[t] = ex;
    __syncthreads();
    if (t == 0) {
        Y run = one;
        int re = 0;
        for (int q = (int)blockDim.x - 1; q >= 0; --q) {
            Y v = sm[q];
            int ve = se[q];
            sm[q] = run;
            se[q] = re;
            run = mul(run, v);
            re += ve;
            normalise(run, re);
        }
    }
    __syncthreads();
    m = sm[t];
    ex = se[t];
    for (int64_t j = c1 - 1; j >= c0; --j) {
        if (j + 1 < n) { m = mul(m, neg(div(one, e[j]))); normalise(m, ex); }
        Q[blk.row0 + j] = m;
        Qe[blk.row0 + j] = ex;
        if (Q64) Q64[blk.row0 + j] = hi_of(m);
    }
}

// ---------------------------------------------------------------------------
// a3: multisection on Sturm counts (L lanes per slot, groups inside a wave)
// ---------------------------------------------------------------------------
template <int L, int PTS>
__global__ void __launch_bounds__(256)
k_bisect(const int64_t* __restrict__ list, int64_t count, Slot* __restrict__ slots,
         const Node* __restrict__ nodes, const Block* __restrict__ blocks,
         const double* __restrict__ d64, const double* __restrict__ lld64, double rtol,
         double widen, double* __restrict__ work, int64_t skip_n) {
    constexpr int G = 256 / L;
    const int g = threadIdx.x / L;
    const int q = threadIdx.x % L;
    const int64_t idx = (int64_t)blockIdx.x * G + g;
    bool active = idx < count;
    int64_t s = 0, n = 0, j = 0;
    double lo = 0.0, hi = 0.0;
    const double* D = d64;
    const double* LL = lld64;
    if (active) {
        s = list[idx];
        const Slot sl = slots[s];
        const Node nd = nodes[sl.node];
        n = blocks[nd.block].n;
        D = d64 + nd.rep;
        LL = lld64 + nd.rep;
        j = sl.idx;
        lo = sl.lo;
        hi = sl.hi;
        // slots of nodes this long are served by the staged kernel
        if (n >= skip_n) {
            active = false;
            n = 0;
        }
    }
    const int lane = threadIdx.x & 63;
    const int gbase = lane - q;  // first lane of this group within the wave
    // make sure the bracket holds: count(lo) <= j-1 < count(hi)
    bool fix = active;
    for (int it = 0; it < 64; ++it) {
        int cl = 0, ch = 0;
        if (fix) {
            if (q == 0) cl = negcount64(D, LL, n, lo);
            if (q == 1 || L == 1) ch = negcount64(D, LL, n, hi);
        }
        // share within the group
        const int cl0 = __shfl(cl, gbase, 64);
        const int ch0 = (L == 1) ? ch : __shfl(ch, gbase + 1, 64);
        bool okb = !fix || (cl0 <= j - 1 && ch0 >= j);
        if (fix && !okb) {
            const double w = fmax(hi - lo, fmax(fabs(lo), fabs(hi)) * 1e-15) + 1e-300;
            if (cl0 > j - 1) lo -= w;
            if (ch0 < j) hi += w;
        }
        fix = fix && !okb;
        if (!__any(fix)) break;
    }
    // multisection until the relative width reaches rtol
    const double lo0 = lo, hi0 = hi;
    bool busy = active;
    int passes = 0;
    for (int it = 0; it < 400; ++it) {
        if (busy) {
            const double w = hi - lo;
            const double scale = fmax(fabs(lo), fabs(hi));
            if (w <= rtol * scale || w <= 1e-300 || !(w > 0.0)) busy = false;
        }
        if (!__any(busy)) break;
        passes += busy ? 1 : 0;
        // L lanes x PTS points: point t = q*PTS + p sits at lo + (t+1) h
        constexpr int NP = L * PTS;
        const double h = (hi - lo) / (double)(NP + 1);
        double xs[PTS];
        int cs[PTS];
#pragma unroll
        for (int p = 0; p < PTS; ++p) xs[p] = lo + h * (double)(q * PTS + p + 1);
        if (busy) {
            negcount64_multi<PTS>(D, LL, n, xs, cs);
        } else {
#pragma unroll
            for (int p = 0; p < PTS; ++p) cs[p] = 0;
        }
        int fp = PTS;  // first of this lane's points with count >= j
#pragma unroll
        for (int p = PTS - 1; p >= 0; --p)
            if (cs[p] >= j) fp = p;
        const unsigned long long m = __ballot(busy && fp < PTS);
        const unsigned long long gm = (m >> gbase) & ((L == 64) ? ~0ull : ((1ull << L) - 1ull));
        const int fq = gm ? __builtin_ctzll(gm) : L;      // first lane with a crossing
        const int fpo = __shfl(fp, gbase + (fq < L ? fq : 0), 64);  // all lanes take part
        if (busy) {
            const int f = (fq < L) ? fq * PTS + fpo : NP;  // first point with count >= j
            const double nlo = (f > 0) ? lo + h * (double)f : lo;
            const double nhi = (f < NP) ? lo + h * (double)(f + 1) : hi;
            if (nlo == lo && nhi == hi) busy = false;
            lo = nlo;
            hi = nhi;
        }
    }
    if (active && q == 0) {
        // algorithmic work: halvings plain bisection needs for this bracket
        const double bits = log2(fmax((lo0 - hi0 == 0.0) ? 1.0 : (hi0 - lo0) / fmax(hi - lo, 1e-300), 1.0));
        atomicAdd(&work[0], bits * (double)n);
        // diagnostics: largest and total number of multisection passes
        atomicMax(reinterpret_cast<unsigned long long*>(&work[6]),
                  (unsigned long long)__double_as_longlong((double)passes));
        atomicAdd(&work[7], (double)passes);
        const double w = widen * (double)n * fmax(fabs(lo), fabs(hi));
        slots[s].lo = lo - w;
        slots[s].hi = hi + w;
    }
}

// ---------------------------------------------------------------------------
// a3 with the representation staged through LDS.  Every workgroup serves
// intervals of one node; the node's rows stream through a double-buffered LDS
// window (one coalesced row load per thread per window, issued a whole window
// ahead), and all counts of the workgroup read each row from LDS as a
// broadcast.  The sequential recurrences then never wait on memory.
// ---------------------------------------------------------------------------
struct BisWG {
    int64_t begin;  // first position in the slot list
    int count;      // intervals served (<= 256 / L)
    int node;
};


// Sturm counts at P shifts for every thread of the workgroup.  All threads
// call it (it synchronises the workgroup); threads with on == false only load.
template <int P>
__device__ __forceinline__ void staged_counts(const double* __restrict__ D,
                                              const double* __restrict__ LL, int64_t n,
                                              const double (&x)[P], int (&neg)[P], bool on,
                                              double2 (*win)[STAGE_ROWS]) {
    const int t = threadIdx.x;
    double a[P], b[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        a[p] = -x[p];
        b[p] = 1.0;
        neg[p] = 0;
    }
    // a workgroup of W threads loads STAGE_ROWS / W rows per thread
    constexpr int RPT = STAGE_ROWS / 64;  // rows per thread, at most (W = 64)
    const int W = blockDim.x;
    for (int j = 0; j < RPT; ++j) {
        const int rr = t + j * W;
        if (rr < STAGE_ROWS && rr < n) win[0][rr] = make_double2(D[rr], LL[rr]);
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 < n; c0 += STAGE_ROWS) {
        const int cur = (int)((c0 / STAGE_ROWS) & 1);
        // next window: loaded now, stored after this window is processed
        double2 nx[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int64_t nr = c0 + STAGE_ROWS + t + j * W;
            nx[j] = make_double2(0.0, 0.0);
            if (t + j * W < STAGE_ROWS && nr < n) nx[j] = make_double2(D[nr], LL[nr]);
        }
        const int64_t left = n - c0;
        if (on) {
            if (left >= STAGE_ROWS) {
                for (int i = 0; i < STAGE_ROWS; i += 8) {
                    double2 r[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) r[u] = win[cur][i + u];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const double c = __fma_rn(r[u].x, b[p], a[p]);
                            neg[p] += sign_differs(c, b[p]);
                            a[p] = __fma_rn(-x[p], c, r[u].y * a[p]);
                            b[p] = c;
                        }
                        if ((u & 3) == 3) {
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                const int em = max(dexp(a[p]), dexp(b[p]));
                                a[p] = __builtin_ldexp(a[p], -em);
                                b[p] = __builtin_ldexp(b[p], -em);
                            }
                        }
                    }
                }
            } else {
                for (int i = 0; i < (int)left; ++i) {
                    const double2 r = win[cur][i];
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const double c = __fma_rn(r.x, b[p], a[p]);
                        neg[p] += sign_differs(c, b[p]);
                        a[p] = __fma_rn(-x[p], c, r.y * a[p]);
                        b[p] = c;
                    }
                    if ((i & 3) == 3) {
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const int em = max(dexp(a[p]), dexp(b[p]));
                            a[p] = __builtin_ldexp(a[p], -em);
                            b[p] = __builtin_ldexp(b[p], -em);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < RPT; ++j)
            if (t + j * W < STAGE_ROWS) win[cur ^ 1][t + j * W] = nx[j];
        __syncthreads();
    }
}

// Sturm counts at P shifts from rows already resident in LDS (nodes of at
// most RESIDENT_ROWS rows stay there for all passes of a workgroup, which
// then needs no barrier and no global load per pass).
constexpr int RESIDENT_ROWS = 4 * STAGE_ROWS;
template <int P>
__device__ __forceinline__ void resident_counts(const double2* __restrict__ rows, int n,
                                                const double (&x)[P], int (&neg)[P], bool on) {
    double a[P], b[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        a[p] = -x[p];
        b[p] = 1.0;
        neg[p] = 0;
    }
    if (!on) return;
    auto step = [&](const double2& r) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double c = __fma_rn(r.x, b[p], a[p]);
            neg[p] += sign_differs(c, b[p]);
            a[p] = __fma_rn(-x[p], c, r.y * a[p]);
            b[p] = c;
        }
    };
    auto rescale = [&]() {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int em = max(dexp(a[p]), dexp(b[p]));
            a[p] = __builtin_ldexp(a[p], -em);
            b[p] = __builtin_ldexp(b[p], -em);
        }
    };
    int i = 0;
    for (; i + 8 <= n; i += 8) {
        double2 r[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) r[u] = rows[i + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) step(r[u]);
        rescale();
#pragma unroll
        for (int u = 4; u < 8; ++u) step(r[u]);
        rescale();
    }
    for (; i < n; ++i) {
        step(rows[i]);
        if ((i & 3) == 3) rescale();
    }
}

template <int L, int PTS>
__global__ void __launch_bounds__(256)
k_bisect_staged(const BisWG* __restrict__ wgs, const int64_t* __restrict__ list,
                Slot* __restrict__ slots, const Node* __restrict__ nodes,
                const Block* __restrict__ blocks, const double* __restrict__ d64,
                const double* __restrict__ lld64, double rtol, double widen,
                double* __restrict__ work, int check) {
    // the staging window, or the whole node when it has at most RESIDENT_ROWS rows
    __shared__ double2 win[RESIDENT_ROWS / STAGE_ROWS][STAGE_ROWS];
    const BisWG w = wgs[blockIdx.x];
    // groups of L lanes never straddle a wave: 64 / L groups per wave (the
    // last 64 mod L lanes of a wave only help with the loads)
    constexpr int GW = 64 / L;
    const int lane = threadIdx.x & 63;
    const int lg = lane / L;
    const int q = lane % L;
    const int g = (threadIdx.x >> 6) * GW + lg;
    const bool active = lg < GW && g < w.count;
    const Node nd = nodes[w.node];
    const int64_t n = blocks[nd.block].n;
    const double* D = d64 + nd.rep;
    const double* LL = lld64 + nd.rep;
    int64_t s = 0, j = 0;
    double lo = 0.0, hi = 0.0;
    if (active) {
        s = list[w.begin + g];
        const Slot sl = slots[s];
        j = sl.idx;
        lo = sl.lo;
        hi = sl.hi;
    }
    const int gbase = (lg < GW ? lg : 0) * L;  // first lane of this group
    // small nodes: all rows resident in the (flattened) window
    const bool resident = n <= RESIDENT_ROWS;
    double2* rows = &win[0][0];
    if (resident) {
        for (int i = threadIdx.x; i < (int)n; i += blockDim.x) rows[i] = make_double2(D[i], LL[i]);
        __syncthreads();
    }
    // make sure the bracket holds: count(lo) <= j-1 < count(hi) (skipped when
    // the caller has verified every bracket with counts already)
    bool fix = active && check;
    for (int it = 0; it < 64; ++it) {
        if (!__syncthreads_or(fix)) break;
        const double xs2[2] = {lo, hi};
        int c2[2];
        if (resident) resident_counts<2>(rows, (int)n, xs2, c2, fix && q == 0);
        else staged_counts<2>(D, LL, n, xs2, c2, fix && q == 0, win);
        const int cl0 = __shfl(c2[0], gbase, 64);
        const int ch0 = __shfl(c2[1], gbase, 64);
        const bool okb = !fix || (cl0 <= j - 1 && ch0 >= j);
        if (fix && !okb) {
            const double wd = fmax(hi - lo, fmax(fabs(lo), fabs(hi)) * 1e-15) + 1e-300;
            if (cl0 > j - 1) lo -= wd;
            if (ch0 < j) hi += wd;
        }
        fix = fix && !okb;
    }
    const double lo0 = lo, hi0 = hi;
    bool busy = active;
    int passes = 0;
    for (int it = 0; it < 400; ++it) {
        if (busy) {
            const double wd = hi - lo;
            const double scale = fmax(fabs(lo), fabs(hi));
            if (wd <= rtol * scale || wd <= 1e-300 || !(wd > 0.0)) busy = false;
        }
        if (!__syncthreads_or(busy)) break;
        passes += busy ? 1 : 0;
        constexpr int NP = L * PTS;
        const double h = (hi - lo) / (double)(NP + 1);
        double xs[PTS];
        int cs[PTS];
#pragma unroll
        for (int p = 0; p < PTS; ++p) xs[p] = lo + h * (double)(q * PTS + p + 1);
        if (resident) resident_counts<PTS>(rows, (int)n, xs, cs, busy);
        else staged_counts<PTS>(D, LL, n, xs, cs, busy, win);
        int fp = PTS;
#pragma unroll
        for (int p = PTS - 1; p >= 0; --p)
            if (cs[p] >= j) fp = p;
        const unsigned long long m = __ballot(busy && fp < PTS);
        const unsigned long long gm = (m >> gbase) & ((L == 64) ? ~0ull : ((1ull << L) - 1ull));
        const int fq = gm ? __builtin_ctzll(gm) : L;
        const int fpo = __shfl(fp, gbase + (fq < L ? fq : 0), 64);
        if (busy) {
            const int f = (fq < L) ? fq * PTS + fpo : NP;
            const double nlo = (f > 0) ? lo + h * (double)f : lo;
            const double nhi = (f < NP) ? lo + h * (double)(f + 1) : hi;
            if (nlo == lo && nhi == hi) busy = false;
            lo = nlo;
            hi = nhi;
        }
    }
    if (active && q == 0) {
        const double bits = log2(fmax((lo0 - hi0 == 0.0) ? 1.0 : (hi0 - lo0) / fmax(hi - lo, 1e-300), 1.0));
        atomicAdd(&work[0], bits * (double)n);
        // diagnostics: largest and total number of multisection passes
        atomicMax(reinterpret_cast<unsigned long long*>(&work[6]),
                  (unsigned long long)__double_as_longlong((double)passes));
        atomicAdd(&work[7], (double)passes);
        const double wd = widen * (double)n * fmax(fabs(lo), fabs(hi));
        slots[s].lo = lo - wd;
        slots[s].hi = hi + wd;
    }
}

// ---------------------------------------------------------------------------
// a3 alternative for whole spectra: the dqds algorithm, the sequential choice
// when every eigenpair of a matrix is wanted (Sec. 4.1), one lane per root.
// The definite root M = L D L^T has the qd array q_k = d_k, e_k = lld_k,
// negated for a negative definite root so that every entry is positive.  The
// differential qd transform with shift s,
//     d = q_0 - s;   qh_k = d + e_k,  t = q_{k+1} / qh_k,  eh_k = e_k t,
//                    d = d t - s;     qh_{m-1} = d,
// gives the qd array of the same matrix shifted by s (factors in the other
// order); all its entries stay positive exactly when s is below the smallest
// eigenvalue.  The shift is Laguerre's step from below for the characteristic
// polynomial of the m x m array,
//     s = m / (S1 + sqrt((m - 1)(m S2 - S1^2))),  S1 = tr A^{-1},  S2 = tr A^{-2},
// which never passes the smallest eigenvalue and converges cubically.  The
// diagonal of A^{-1} is 1/g_k, g_k the twist elements at zero shift, and S2 is
// the derivative of S1 with respect to the shift: with the top-down values
// u_0 = -1, u_{k+1} = (e_k / q_k) u_k - 1 (derivatives of the stationary
// transform) and the bottom-up p_{m-1} = q_{m-1}, p_k = p_{k+1} q_k / r_k,
// r_k = e_k + p_{k+1}, with derivatives v_{m-1} = -1,
// v_k = q_k e_k v_{k+1} / r_k^2 - 1, one has g_k = p_k and
// g_k' = u_k + v_k + 1, so S1 = sum 1/g_k and S2 = -sum g_k' / g_k^2.  The
// u_k of the next array are formed inside the transform.  A transform that
// fails anyway (rounding) is retried with smaller shifts, down to zero, which
// cannot fail.  The bottom entry deflates when e_{m-2} is small enough that
// dropping it moves the eigenvalue by at most about a unit roundoff (the
// singular values of the bidiagonal factor move by at most sqrt(e_{m-2}));
// the bottom 2 x 2 block deflates likewise on e_{m-3}, which settles close
// pairs without resolving them by shifts.  The values come out nearly
// ascending and an insertion sort orders them.  They are estimates only: the
// multisection that follows checks every bracket with Sturm counts, repairs
// it where needed and refines it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool dqds_deflates(double lam, double sh, double el) {
    const double tol = 1.1102230246251565e-16 * (sh + lam);
    return el <= tol && 4.0 * lam * el <= tol * tol;
}

__global__ void __launch_bounds__(64)
k_dqds(const int* __restrict__ blist, int count, const Block* __restrict__ blocks,
       const Node* __restrict__ nodes, const double* __restrict__ d64,
       const double* __restrict__ lld64, double* __restrict__ scratch, Slot* __restrict__ slots,
       unsigned long long* __restrict__ transforms) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= count) return;
    const int b = blist[i];
    const Block bk = blocks[b];
    const int64_t n = bk.n;
    const Node nd = nodes[b];  // root node of block b
    const double* D = d64 + nd.rep;
    const double* LL = lld64 + nd.rep;
    // six arrays of n per root: the qd array and its transform, u, the values
    double* q = scratch + 6 * bk.row0;
    double* e = q + n;
    double* q2 = e + n;
    double* e2 = q2 + n;
    double* u = e2 + n;
    double* ev = u + n;
    const double sg = (n > 0 && D[0] < 0.0) ? -1.0 : 1.0;  // a definite root: one sign
    double uk = -1.0;
    for (int64_t k = 0; k < n; ++k) {
        q[k] = sg * D[k];
        e[k] = (k + 1 < n) ? sg * LL[k] : 0.0;
        u[k] = uk;
        uk = (e[k] / q[k]) * uk - 1.0;
    }
    constexpr double EPS = 1.1102230246251565e-16;
    double sh = 0.0, sl = 0.0;  // accumulated shift (compensated sum)
    int64_t m = n, found = 0;
    unsigned long long steps = 0;
    int64_t budget = 12 * n + 40;  // transforms before giving up on the rest
    while (m > 0) {
        if (m == 1) {
            ev[found++] = sh + (sl + q[0]);
            m = 0;
            break;
        }
        if (dqds_deflates(q[m - 1], sh, e[m - 2])) {
            ev[found++] = sh + (sl + q[m - 1]);
            --m;
            continue;
        }
        {
            // bottom 2 x 2 block: [[a, sqrt(a b)], [sqrt(a b), b + c]]
            const double a = q[m - 2], bb = e[m - 2], c = q[m - 1];
            const double tr2 = a + bb + c;
            const double big = 0.5 * (tr2 + sqrt(fmax(tr2 * tr2 - 4.0 * a * c, 0.0)));
            const double small = a * c / big;
            if (m == 2 || dqds_deflates(small, sh, e[m - 3])) {
                ev[found++] = sh + (sl + small);
                ev[found++] = sh + (sl + big);
                m -= 2;
                continue;
            }
        }
        if (budget-- <= 0) break;
        // Laguerre shift from S1 = tr A^{-1}, S2 = tr A^{-2}
        double p = q[m - 1], v = -1.0;
        double S1, S2;
        {
            const double ip = 1.0 / p;
            S1 = ip;
            S2 = -(u[m - 1] + v + 1.0) * ip * ip;
        }
        auto up = [&](double qk, double ek, double uk) {
            const double rr = 1.0 / (ek + p);
            v = __fma_rn(qk * ek * v, rr * rr, -1.0);
            p = p * qk * rr;
            const double ip = 1.0 / p;
            S1 += ip;
            S2 -= (uk + v + 1.0) * ip * ip;
        };
        int64_t k = m - 2;
        for (; k >= 7; k -= 8) {  // loads of a block of rows first
            double qk[8], ek[8], uk[8];
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                qk[w] = q[k - w];
                ek[w] = e[k - w];
                uk[w] = u[k - w];
            }
#pragma unroll
            for (int w = 0; w < 8; ++w) up(qk[w], ek[w], uk[w]);
        }
        for (; k >= 0; --k) up(q[k], e[k], u[k]);
        const double fm = (double)m;
        double s = fm / (S1 + sqrt(fmax((fm - 1.0) * (fm * S2 - S1 * S1), 0.0)));
        s *= 1.0 - 8.0 * fm * EPS;
        if (!(s > 0.0) || !isfinite(s)) s = 0.0;
        bool ok = false;
        for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
            if (attempt == 3) s = 0.0;
            else if (attempt > 0) s *= 0.25;
            double d = q[0] - s;
            double un = -1.0;
            ok = d > 0.0;
            auto row = [&](int64_t j, double qn, double ej) {
                const double rq = 1.0 / (d + ej);
                const double t = qn * rq;
                const double eh = ej * t;
                q2[j] = d + ej;
                e2[j] = eh;
                u[j] = un;
                un = __fma_rn(eh * rq, un, -1.0);
                d = __fma_rn(d, t, -s);
                ok = ok && d > 0.0;
            };
            int64_t j = 0;
            for (; j + 8 < m && ok; j += 8) {  // a failed block is discarded with the rest
                double qn[8], ej[8];
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    qn[w] = q[j + 1 + w];
                    ej[w] = e[j + w];
                }
#pragma unroll
                for (int w = 0; w < 8; ++w) row(j + w, qn[w], ej[w]);
            }
            for (; j + 1 < m && ok; ++j) row(j, q[j + 1], e[j]);
            q2[m - 1] = d;
            u[m - 1] = un;
            ++steps;
        }
        if (!ok) break;
        double* tq = q;
        q = q2;
        q2 = tq;
        double* te = e;
        e = e2;
        e2 = te;
        const double x = sh + s, bv = x - sh;
        sl += (sh - (x - bv)) + (s - bv);
        sh = x;
    }
    // an unfinished array leaves rough estimates; the bracket check repairs them
    for (int64_t k = 0; k < m; ++k) ev[found++] = sh + (sl + q[k]);
    for (int64_t k = 1; k < n; ++k) {
        const double val = ev[k];
        int64_t j = k - 1;
        while (j >= 0 && ev[j] > val) {
            ev[j + 1] = ev[j];
            --j;
        }
        ev[j + 1] = val;
    }
    const double w0 = 4.0 * (double)n * EPS;
    for (int64_t k = 0; k < bk.nslot; ++k) {
        const int64_t sidx = bk.slot0 + k;
        const int64_t j = slots[sidx].idx;  // 1-based index among the eigenvalues of M
        const double lam = (sg > 0.0) ? ev[j - 1] : -ev[n - j];
        const double w = w0 * fabs(lam) + 1e-300;
        slots[sidx].lo = lam - w;
        slots[sidx].hi = lam + w;
    }
    atomicAdd(transforms, steps);
}

// ---------------------------------------------------------------------------
// Spectrum slicing before the per-eigenvalue multisection of a large root:
// Sturm counts at M equally spaced interior points of the root interval are
// shared by all eigenvalues of the block, so every eigenvalue starts from one
// slice of width (hi - lo) / (M + 1) -- log2(M + 1) bisection steps for the
// price of M counts.  Brackets are taken only where the counts prove them.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double slice_point(double lo, double hi, int64_t m, int64_t M) {
    return lo + (hi - lo) * ((double)(m + 1) / (double)(M + 1));
}

__global__ void __launch_bounds__(256)
k_slice(const Block* __restrict__ blocks, int b, const Node* __restrict__ nodes,
        const Slot* __restrict__ slots, const double* __restrict__ d64,
        const double* __restrict__ lld64, int64_t M, int* __restrict__ cnt) {
    __shared__ double2 win[2][STAGE_ROWS];
    const Block blk = blocks[b];
    const Node nd = nodes[b];
    const double lo = slots[blk.slot0].lo, hi = slots[blk.slot0].hi;
    const int64_t m = (int64_t)blockIdx.x * STAGE_ROWS + threadIdx.x;  // M is a multiple
    const double xs[1] = {slice_point(lo, hi, m, M)};
    int c[1];
    staged_counts<1>(d64 + nd.rep, lld64 + nd.rep, blk.n, xs, c, true, win);
    cnt[m] = c[0];
    // the root interval, for k_slice_assign (which rewrites the slots)
    if (m == 0) {
        reinterpret_cast<double*>(cnt + M)[0] = lo;
        reinterpret_cast<double*>(cnt + M)[1] = hi;
    }
}

__global__ void __launch_bounds__(256)
k_slice_assign(const Block* __restrict__ blocks, int b, Slot* __restrict__ slots, int64_t M,
               const int* __restrict__ cnt, double* __restrict__ work) {
    const Block blk = blocks[b];
    const int64_t s = blk.slot0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= blk.slot0 + blk.nslot) return;
    // the root interval as k_slice saw it (slots[slot0] may already be rewritten
    // by another workgroup of this launch)
    const double lo = reinterpret_cast<const double*>(cnt + M)[0];
    const double hi = reinterpret_cast<const double*>(cnt + M)[1];
    const int64_t j = slots[s].idx;
    // first point whose count reaches j
    int64_t a = 0, z = M;
    while (a < z) {
        const int64_t mid = (a + z) >> 1;
        if (cnt[mid] >= j) z = mid;
        else a = mid + 1;
    }
    const bool ok = (a == M || cnt[a] >= j) && (a == 0 || cnt[a - 1] <= j - 1);
    if (!ok) return;  // counts not monotone here: keep the root interval
    const double nlo = (a == 0) ? lo : slice_point(lo, hi, a - 1, M);
    const double nhi = (a == M) ? hi : slice_point(lo, hi, a, M);
    slots[s].lo = nlo;
    slots[s].hi = nhi;
    // algorithmic work: the halvings plain bisection needs for this narrowing
    atomicAdd(&work[0], log2((hi - lo) / fmax(nhi - nlo, 1e-300)) * (double)blk.n);
}

// Spectrum slicing of small roots (at most RESIDENT_ROWS rows), one workgroup
// per root: the rows stay in LDS, and M counts at equally spaced points of the
// root interval are shared by the root's eigenvalues.  M is the power of two
// from 64 to SLICE_SMALL_MAX that is at least twice the wanted eigenvalues, and
// each eigenvalue takes the slice its counts prove, as with k_slice and
// k_slice_assign for large roots (a bracket the counts do not prove keeps the
// root interval).
constexpr int SLICE_SMALL_MAX = 2048;

__global__ void __launch_bounds__(256)
k_slice_small(const int* __restrict__ blist, const Block* __restrict__ blocks,
              const Node* __restrict__ nodes, Slot* __restrict__ slots,
              const double* __restrict__ d64, const double* __restrict__ lld64,
              double* __restrict__ work) {
    __shared__ double2 rows[RESIDENT_ROWS];
    __shared__ int cnt[SLICE_SMALL_MAX];
    __shared__ double s_lo, s_hi;
    const int b = blist[blockIdx.x];
    const Block blk = blocks[b];
    const Node nd = nodes[b];
    const int n = (int)blk.n;  // at most RESIDENT_ROWS (the host's choice)
    const int t = threadIdx.x;
    int M = 64;
    while (M < 2 * blk.nslot && M < SLICE_SMALL_MAX) M *= 2;
    // every slot of the root starts from the root interval
    if (t == 0) {
        s_lo = slots[blk.slot0].lo;
        s_hi = slots[blk.slot0].hi;
    }
    for (int i = t; i < n; i += blockDim.x) rows[i] = make_double2(d64[nd.rep + i], lld64[nd.rep + i]);
    __syncthreads();
    const double lo = s_lo, hi = s_hi;
    for (int m = t; m < M; m += blockDim.x) {
        const double xs[1] = {slice_point(lo, hi, m, M)};
        int c[1];
        resident_counts<1>(rows, n, xs, c, true);
        cnt[m] = c[0];
    }
    __syncthreads();
    for (int64_t s = blk.slot0 + t; s < blk.slot0 + blk.nslot; s += blockDim.x) {
        const int64_t j = slots[s].idx;
        // first point whose count reaches j
        int a = 0, z = M;
        while (a < z) {
            const int mid = (a + z) >> 1;
            if (cnt[mid] >= j) z = mid;
            else a = mid + 1;
        }
        const bool ok = (a == M || cnt[a] >= j) && (a == 0 || cnt[a - 1] <= j - 1);
        if (!ok) continue;  // counts not monotone here: keep the root interval
        const double nlo = (a == 0) ? lo : slice_point(lo, hi, a - 1, M);
        const double nhi = (a == M) ? hi : slice_point(lo, hi, a, M);
        slots[s].lo = nlo;
        slots[s].hi = nhi;
        // algorithmic work: the halvings plain bisection needs for this narrowing
        atomicAdd(&work[0], log2((hi - lo) / fmax(nhi - nlo, 1e-300)) * (double)n);
    }
}

// ---------------------------------------------------------------------------
// Verification of binary64-copy intervals in working precision y (Sec. 3.2:
// results of x-bit eigenvalue computations may be verified or refined in y).
// Two lanes per slot count the y representation at lo and hi; a bracket that
// does not hold for the y representation is widened until it does and then
// refined by bisection in y to relative width rtol.  With refine_all every
// bracket is refined that way (the binary64 copy does not resolve gaptol:
// (k_rr + k_bi) n eps_x > gaptol).
// ---------------------------------------------------------------------------
// Sturm count in y at x for threads with on == true; the node's rows stream
// through an LDS window filled by the 64 threads of the workgroup (all call).
template <class Y>
__device__ __forceinline__ int staged_count_y(const Y* __restrict__ D, const Y* __restrict__ LL,
                              const Y* __restrict__ E, int64_t n, Y x,
                              bool on, Y (*wd)[STAGE_ROWS], Y (*wl)[STAGE_ROWS]) {
    constexpr int PER = STAGE_ROWS / 64;
    const int t = threadIdx.x;
    Y a = neg(x), b = y_from(1.0, Y());
    int negc = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = t + 64 * k;
        if (i < n) {
            wd[0][t + 64 * k] = D[i];
            wl[0][t + 64 * k] = lld_at(LL, E, D, i, n);
        }
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 < n; c0 += STAGE_ROWS) {
        const int cur = (int)((c0 / STAGE_ROWS) & 1);
        Y nd[PER], nl[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t i = c0 + STAGE_ROWS + t + 64 * k;
            nd[k] = (i < n) ? D[i] : y_from(0.0, Y());
            nl[k] = (i < n) ? lld_at(LL, E, D, i, n) : y_from(0.0, Y());
        }
        if (on) {
            const int cnt = (int)min<int64_t>(STAGE_ROWS, n - c0);
            auto row = [&](const Y& dv, const Y& lv, int i) {
                const Y c = mul_add(dv, b, a);
                negc += sign_differs(hi_of(c), hi_of(b));
                a = mul_sub(lv, a, x, c);
                b = c;
                if ((i & 3) == 3) {
                    const int em = max(y_exp(a), y_exp(b));
                    a = y_ldexp(a, -em);
                    b = y_ldexp(b, -em);
                }
            };
            int i = 0;
            for (; i + 8 <= cnt; i += 8) {
                Y dv[8], lv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    dv[u] = wd[cur][i + u];
                    lv[u] = wl[cur][i + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) row(dv[u], lv[u], i + u);
            }
            for (; i < cnt; ++i) row(wd[cur][i], wl[cur][i], i);
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            wd[cur ^ 1][t + 64 * k] = nd[k];
            wl[cur ^ 1][t + 64 * k] = nl[k];
        }
        __syncthreads();
    }
    return negc;
}

// One workgroup of 64 threads serves up to 32 slots of one node (wgs[]); two
// lanes per slot count at lo and at hi.
template <class Y>
__global__ void __launch_bounds__(64)
k_verify(const BisWG* __restrict__ wgs, const int64_t* __restrict__ list, Slot* __restrict__ slots,
         const Node* __restrict__ nodes, const Block* __restrict__ blocks,
         const Y* __restrict__ rep_d, const Y* __restrict__ rep_lld, const Y* __restrict__ rep_e,
         double rtol, unsigned long long* __restrict__ repaired, int refine_all) {
    __shared__ Y wd[2][STAGE_ROWS], wl[2][STAGE_ROWS];
    const BisWG w = wgs[blockIdx.x];
    const int lane = threadIdx.x;
    const int pair = lane >> 1;
    const bool side = lane & 1;  // 0: count at lo, 1: count at hi
    const bool active = pair < w.count;
    const Node nd = nodes[w.node];
    const int64_t n = blocks[nd.block].n;
    const Y* D = rep_d + nd.rep;
    const Y* LL = rep_lld ? rep_lld + nd.rep : nullptr;
    const Y* E = rep_e + blocks[nd.block].row0;
    int64_t s = 0, j = 0;
    double lo = 0, hi = 0;
    if (active) {
        s = list[w.begin + pair];
        const Slot sl = slots[s];
        j = sl.idx;
        lo = sl.lo;
        hi = sl.hi;
    }
    bool bad = false, fix = active;
    for (int it = 0; it < 80; ++it) {
        if (!__syncthreads_or(fix)) break;
        const int c = staged_count_y<Y>(D, LL, E, n, y_from(side ? hi : lo, Y()), fix, wd, wl);
        const int co = __shfl_xor(c, 1, 64);
        const int clo = side ? co : c, chi = side ? c : co;
        if (fix) {
            const bool ok = (clo <= j - 1) && (chi >= j);
            if (!ok) {
                bad = true;
                const double wdt = fmax(hi - lo, fmax(fabs(lo), fabs(hi)) * 1e-14) + 1e-300;
                if (clo > j - 1) lo -= wdt;
                if (chi < j) hi += wdt;
            }
            fix = !ok;
        }
    }
    // refine repaired brackets (or all) by bisection in y (two points per step)
    bool busy = bad || (refine_all && active);
    for (int it = 0; it < 200; ++it) {
        if (busy) {
            const double wdt = hi - lo;
            if (!(wdt > rtol * fmax(fabs(lo), fabs(hi))) || wdt <= 1e-300) busy = false;
        }
        if (!__syncthreads_or(busy)) break;
        const double h3 = (hi - lo) / 3.0;
        const double x = side ? lo + 2.0 * h3 : lo + h3;
        const int c = staged_count_y<Y>(D, LL, E, n, y_from(x, Y()), busy, wd, wl);
        const int co = __shfl_xor(c, 1, 64);
        if (busy) {
            const int c1 = side ? co : c, c2 = side ? c : co;
            const double x1 = lo + h3, x2 = lo + 2.0 * h3;
            if (c1 >= j) hi = x1;
            else if (c2 >= j) { lo = x1; hi = x2; }
            else lo = x2;
        }
    }
    if (active && !side && (bad || refine_all)) {
        slots[s].lo = lo;
        slots[s].hi = hi;
        if (bad) atomicAdd(repaired, 1ull);
    }
}

// ---------------------------------------------------------------------------
// a4: classification (one workgroup per node)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double reldist(const Slot& a, const Slot& b) {
    const double den = fmax(fmax(fabs(a.lo), fabs(a.hi)), fmax(fabs(b.lo), fabs(b.hi)));
    if (den == 0.0) return MR3_BIG;
    return (b.lo - a.hi) / den;
}

__global__ void __launch_bounds__(256)
k_classify(const int64_t* __restrict__ node_list, int64_t count, const Node* __restrict__ nodes,
           Slot* __restrict__ slots, int* __restrict__ start_flag, double gaptol, double gaptol_abs,
           int force_single) {
    const int64_t ni = node_list[blockIdx.x];
    const Node nd = nodes[ni];
    const int t = threadIdx.x;
    for (int64_t s = nd.first + t; s <= nd.last; s += blockDim.x) {
        int f = 1;
        if (s > nd.first && !force_single) {
            // relative separation, amended by the absolute one when enabled
            const Slot a = slots[s - 1], b = slots[s];
            f = reldist(a, b) >= gaptol || (gaptol_abs > 0.0 && b.lo - a.hi >= gaptol_abs * nd.spdiam);
        }
        start_flag[s] = f;
    }
    __syncthreads();
    for (int64_t s = nd.first + t; s <= nd.last; s += blockDim.x) {
        if (!start_flag[s]) continue;
        int64_t e = s;
        while (e < nd.last && !start_flag[e + 1]) ++e;
        bool req = false;
        for (int64_t u = s; u <= e; ++u) req |= (slots[u].out >= 0);
        const double lg = (s > nd.first) ? slots[s].lo - slots[s - 1].hi : slots[s].lgap;
        const double rg = (e < nd.last) ? slots[e + 1].lo - slots[e].hi : slots[e].rgap;
        if (e == s) {
            slots[s].kind = req ? KIND_SINGLETON : KIND_HELPER;
            slots[s].lgap = lg;
            slots[s].rgap = rg;
        } else if (req) {
            slots[s].kind = KIND_CLUSTER_HEAD;
            slots[s].run_end = e;
            slots[s].lgap = lg;
            slots[e].rgap = rg;
            for (int64_t u = s + 1; u <= e; ++u) slots[u].kind = KIND_CLUSTER_MEMBER;
        } else {
            for (int64_t u = s; u <= e; ++u) slots[u].kind = KIND_DROPPED;
        }
    }
}

// ---------------------------------------------------------------------------
// a6: Rayleigh quotient iteration with twisted factorizations
// one wave per 32 singletons; lane 2q sweeps top-down, lane 2q+1 bottom-up
// ---------------------------------------------------------------------------
// Per-lane sweep output.  z is stored in a scaled frame: when a stored value
// would pass about 2^300 the frame is rebased (an "event" at that row).  The
// output kernel multiplies values stored before the last event by ev2f and
// zeroes those stored before the one-but-last, which lie below 2^-300 times
// the growth of z over four rows, relative to the final maximum.  z values are products of the leading parts (binary64
// accuracy, all the output needs).
template <class Y>
struct Half {
    Y sp;        // s_r (top lane) or p_r (bottom lane)
    double zr;   // z at the twist row, in the lane's storage frame
    double ss;   // sum of squares of stored z, storage frame
    double zmax; // largest |stored z| and its row
    int64_t zmaxk;
    int64_t ev1, ev2;  // rebasing events
    double ev2f;
};

// shuffle of a working-precision value between the lanes of a pair
template <class Y>
__device__ __forceinline__ Y shfl_y(Y v, int src);
template <>
__device__ __forceinline__ double shfl_y<double>(double v, int src) { return __shfl(v, src, 64); }
template <>
__device__ __forceinline__ dd shfl_y<dd>(dd v, int src) {
    return mk_dd(__shfl(v.hi, src, 64), __shfl(v.lo, src, 64));
}

// ---------------------------------------------------------------------------
// LDS windows of the RQI sweeps.  All pairs of a chunk belong to one node, so
// at step `it` every top lane reads row it and every bottom lane row n-1-it
// (advancing over row n-2-it).  While a window of SW steps is processed, the
// 64 threads load the next window of both streams, one step of one stream
// each.  In the bottom stream d and lld swap roles, so both lanes run the same
// recurrence: c = f b + a, a' = g a - tau c.
// ---------------------------------------------------------------------------
constexpr int SW = 32;

struct ChunkInfo {
    int64_t begin;  // first position in the singleton list
    int count;      // pairs in the chunk (<= 32), all of one node
    int pad;
};

template <class Y>
struct SweepStep {
    Y pq, f, g;
    int pqe;
};

template <class Y>
struct SweepWin {
    Y pq[2][2][SW];  // [buffer][stream][step]
    Y f[2][2][SW];
    Y g[2][2][SW];
    int pqe[2][2][SW];
};

// DL: lld formed from e and d (nodes without a stored lld); a template
// argument, so that the sweeps of the stored form carry none of its code
template <class Y, bool DL>
__device__ __forceinline__ SweepStep<Y> load_sweep_step(int stream, int64_t it,
                                                        const Y* __restrict__ D,
                                                        const Y* __restrict__ LL,
                                                        const Y* __restrict__ E,
                                                        const Y* __restrict__ P,
                                                        const int* __restrict__ Pe,
                                                        const Y* __restrict__ Q,
                                                        const int* __restrict__ Qe, int64_t n) {
    SweepStep<Y> w;
    if (it >= n) {
        w.pq = w.f = w.g = y_from(0.0, Y());
        w.pqe = 0;
    } else if (stream == 0) {
        w.pq = P[it];
        w.pqe = Pe[it];
        w.f = D[it];
        w.g = DL ? lld_at<Y>(nullptr, E, D, it, n) : LL[it];
    } else {
        // the advance row n-2-it is -1 only on the twist row of r = 0, whose
        // f and g are never used; the pool keeps a guard row there
        const int64_t kz = n - 1 - it, ka = kz - 1;
        w.pq = Q[kz];
        w.pqe = Qe[kz];
        w.f = DL ? lld_at<Y>(nullptr, E, D, ka, n) : LL[ka];
        w.g = D[ka];
    }
    return w;
}

template <class Y>
__device__ __forceinline__ void put_sweep_step(SweepWin<Y>& win, int buf, int stream, int u,
                                               const SweepStep<Y>& w) {
    win.pq[buf][stream][u] = w.pq;
    win.f[buf][stream][u] = w.f;
    win.g[buf][stream][u] = w.g;
    win.pqe[buf][stream][u] = w.pqe;
}

template <class Y>
__device__ __forceinline__ SweepStep<Y> get_sweep_step(const SweepWin<Y>& win, int buf, int stream,
                                                       int u) {
    SweepStep<Y> w;
    w.pq = win.pq[buf][stream][u];
    w.f = win.f[buf][stream][u];
    w.g = win.g[buf][stream][u];
    w.pqe = win.pqe[buf][stream][u];
    return w;
}

// k_rqi<Y, NW> runs NW (1 or RQI_WAVES) independent waves per workgroup, one
// chunk each; the waves of a workgroup share the CU's L1, which pays when
// their chunks sweep the same representation.  The LDS windows are sized for
// NW waves, so one-wave workgroups keep their footprint (and the occupancy
// it allows) to one wave's windows.  A wave synchronises
// only with itself: its lanes exchange data through its own LDS windows and
// its tile.
constexpr int RQI_WAVES = 4;
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// LDS window of the binary64 twist search: the copy's rows of both streams,
// roles swapped in the bottom stream as in the sweeps.
struct TwistWin {
    double f[2][2][SW];  // [buffer][stream][step]
    double g[2][2][SW];
};

// One phase of the binary64 twist search for every lane of the chunk's wave
// (all 64 threads call it).  In this phase stream 0 (top lanes) starts at
// step s0t and stream 1 (bottom lanes) at step s0b; this lane runs cnt steps.
// Step s handles row k = s (top, stationary transform) or k = n-1-s (bottom,
// progressive transform).  Without `combine` the quotient s_k = a/b (resp.
// p_k) is stored in the lane's tile column; with it, the value the other lane
// stored for row k is combined into |gamma_k| = |s_k + p_k + tau| and the
// minimum is tracked.
//
// The phase is bound by memory latency unless its tile traffic is issued well
// ahead: every lane of the wave, active or not, first runs `uni` steps (a
// count for which every lane's rows lie in its own half of its own tile
// column) in whole windows of straight-line code, so that a window's wait for
// the next window's rows counts exactly its SW stores instead of waiting for
// all of them, and the combining phase loads each window's tile values one
// window ahead, each block of 8 replaced once used.  The remaining steps run
// with per-lane counts, reading tile values one block of 8 steps ahead.
// Results of lanes without a pair are never used.
__device__ __forceinline__ void prepass_staged(bool top, const double* __restrict__ D,
                               const double* __restrict__ LL, int64_t n, double tau, int64_t s0t,
                               int64_t s0b, int64_t cnt, int64_t uni, double& a, double& b,
                               bool combine, double* __restrict__ col, double& gmin, int64_t& rmin,
                               TwistWin& win) {
    const int t = threadIdx.x & 63;
    const int side = top ? 0 : 1;
    const int64_t s0 = top ? s0t : s0b;
    int64_t cmax = cnt;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cmax = max(cmax, (int64_t)__shfl_xor(cmax, off, 64));
    auto load = [&](int stream, int64_t o) -> double2 {
        const int64_t sidx = (stream == 0 ? s0t : s0b) + o;
        if (sidx >= n) return make_double2(0.0, 0.0);
        if (stream == 0) return make_double2(D[sidx], LL[sidx]);
        const int64_t ka = n - 2 - sidx;  // advance row of k = n-1-s (guard row at -1)
        return make_double2(LL[ka], D[ka]);
    };
    auto rowk = [&](int64_t o) -> int64_t { return top ? s0 + o : n - 1 - (s0 + o); };
    // lanes without a pair (cnt == 0) run the whole windows too, on one row
    // of their own tile column, so that their accesses stay in the cache
    const bool live = cnt > 0;
    auto rowt = [&](int64_t o) -> int64_t { return live ? rowk(o) : 0; };
    {
        const double2 w = load(t >> 5, t & 31);
        win.f[0][t >> 5][t & 31] = w.x;
        win.g[0][t >> 5][t & 31] = w.y;
    }
    wave_sync();
    // the quotient needs no correct rounding (it only ranks rows): the
    // hardware reciprocal refined by one Newton step is within a few ulps.
    // Ties go to the smallest row: the top lane visits rows upwards and keeps
    // the first minimum, the bottom lane visits them downwards and keeps the
    // last.
    int omin = -1;
    auto step = [&](double f, double g, double ct, int o) {
        double rb = __builtin_amdgcn_rcp(b);
        rb = __fma_rn(__fma_rn(-b, rb, 1.0), rb, rb);
        const double q = a * rb;
        if (combine) {
            const double gv = fabs(q + ct + tau);
            const bool take = top ? (gv < gmin) : (gv <= gmin);
            gmin = take ? gv : gmin;
            omin = take ? o : omin;
        } else {
            col[rowt(o) * 32] = q;
        }
        const double c = __fma_rn(f, b, a);
        a = __fma_rn(-tau, c, g * a);
        b = c;
        if ((o & 3) == 3) {
            const int em = max(dexp(a), dexp(b));
            a = __builtin_ldexp(a, -em);
            b = __builtin_ldexp(b, -em);
        }
    };
    // one whole window at step o0 (a multiple of SW); with `combine` its tile
    // values are in ct, and each block of 8 of them is replaced, once used,
    // by the same block of the next window (a window past the whole ones
    // loads the last of them again, never used).  The next window's rows are
    // loaded meanwhile.
    const int nfw = (int)(uni / SW);
    const int64_t zst = live ? (top ? 32 : -32) : 0;
    auto window = [&](int o0, double (&ct)[SW]) {
        const int cur = (o0 / SW) & 1;
        const double2 nx = load(t >> 5, o0 + SW + (t & 31));
        const double* p = col + rowt(min(o0 + SW, (nfw - 1) * SW)) * 32;
#pragma unroll
        for (int u = 0; u < SW; u += 8) {
            double f[8], g[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                f[v] = win.f[cur][side][u + v];
                g[v] = win.g[cur][side][u + v];
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) step(f[v], g[v], ct[u + v], o0 + u + v);
            if (combine) {
#pragma unroll
                for (int v = 0; v < 8; ++v) ct[u + v] = p[(int64_t)(u + v) * zst];
            }
        }
        win.f[cur ^ 1][t >> 5][t & 31] = nx.x;
        win.g[cur ^ 1][t >> 5][t & 31] = nx.y;
        wave_sync();
    };
    int ob = 0;  // first step of the per-lane remainder
    if (nfw >= 1) {
        double ct[SW];
        if (combine) {
            const double* p = col + rowt(0) * 32;
#pragma unroll
            for (int v = 0; v < SW; ++v) ct[v] = p[(int64_t)v * zst];
        } else {
#pragma unroll
            for (int v = 0; v < SW; ++v) ct[v] = 0.0;
        }
        for (; ob < nfw * SW; ob += SW) window(ob, ct);
    }
    // the remaining steps: per-lane counts, tile values one block of 8 ahead
    double ctn[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) ctn[v] = (combine && ob + v < cnt) ? col[rowk(ob + v) * 32] : 0.0;
    const int icnt = (int)cnt, icmax = (int)cmax;
    for (int o0 = ob; o0 < icmax; o0 += SW) {
        const int cur = (o0 / SW) & 1;
        const double2 nx = load(t >> 5, o0 + SW + (t & 31));
        if (o0 < icnt) {
            const int m = min(SW, icnt - o0);
            int u = 0;
            for (; u + 8 <= m; u += 8) {
                double ctc[8];
#pragma unroll
                for (int v = 0; v < 8; ++v) ctc[v] = ctn[v];
                if (combine) {
#pragma unroll
                    for (int v = 0; v < 8; ++v) {
                        const int o = o0 + u + 8 + v;
                        ctn[v] = (o < icnt) ? col[rowk(o) * 32] : 0.0;
                    }
                }
                double f[8], g[8];
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    f[v] = win.f[cur][side][u + v];
                    g[v] = win.g[cur][side][u + v];
                }
#pragma unroll
                for (int v = 0; v < 8; ++v) step(f[v], g[v], ctc[v], o0 + u + v);
            }
            // tail of the phase (fewer than 8 steps): its tile values are in ctn
            for (int v = 0; u < m; ++u, ++v)
                step(win.f[cur][side][u], win.g[cur][side][u], ctn[v & 7], o0 + u);
        }
        win.f[cur ^ 1][t >> 5][t & 31] = nx.x;
        win.g[cur ^ 1][t >> 5][t & 31] = nx.y;
        wave_sync();
    }
    if (combine && omin >= 0) rmin = rowk(omin);
}

// One sweep of every lane of the chunk's wave (all 64 threads call it; lanes
// with steps == 0 only help with the loads).  The top lane runs the
// stationary transform over rows 0..r, the bottom lane the progressive one
// over rows n-1..r, each storing its part of z in its tile column.  Steps go
// in groups of four: the storage frame is checked on the group's last value
// (and on the twist row), and the pair (a, b) is rescaled after every second
// group.
// Between checks a stored value grows by at most four rows' growth of z, so
// values stay far below overflow (and their squares in ss) for per-row growth
// up to 2^50.  Book-keeping is by step index (32-bit), turned into rows at
// the end.
// (always inlined, like every function here that takes an LDS window: as a
// called function it would reach the window through generic pointers, whose
// accesses also wait for the outstanding global stores)
template <class Y, bool DL>
__device__ __forceinline__ Half<Y> sweep_staged(bool top, const Y* __restrict__ D, const Y* __restrict__ LL,
                                const Y* __restrict__ E,
                                const Y* __restrict__ P, const int* __restrict__ Pe,
                                const Y* __restrict__ Q, const int* __restrict__ Qe, int64_t n,
                                int64_t r, Y tau, double* __restrict__ col, bool store,
                                int64_t steps, SweepWin<Y>& win) {
    const int t = threadIdx.x & 63;
    const int side = top ? 0 : 1;
    Half<Y> h;
    h.zr = 0.0;
    double ss = 0.0, zmax = 0.0;
    int zmi = -1;                        // step of the largest stored |z|
    int ev1 = 0, ev2 = 0, ev2e = 0;      // steps of the last two rebasings, last shift
    Y a = neg(tau), b = y_from(1.0, Y());
    if (!top && steps > 0) a = sub(D[n - 1], tau);
    // binary exponent carried by b, less the storage frame's exponent
    int ebr = 0;
    const int nsteps = (int)steps;
    int smax = nsteps;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) smax = max(smax, __shfl_xor(smax, off, 64));
    double* zp = col + (top ? (int64_t)0 : (n - 1) * 32);  // tile row of the current step
    const int64_t zstep = top ? 32 : -32;
    put_sweep_step<Y>(win, 0, t >> 5, t & 31,
                      load_sweep_step<Y, DL>(t >> 5, t & 31, D, LL, E, P, Pe, Q, Qe, n));
    wave_sync();
    // the value of z at a step, after the storage check when `check`
    auto zvalue = [&](const SweepStep<Y>& w, int it, bool check) -> double {
        const double pb = prod_hi(w.pq, b);
        int ex = w.pqe + ebr;
        if (check) {
            const int ez = dexp(pb) + ex;
            const bool rb = ez > 300;
            const int dlt = rb ? ez : 0;
            ebr -= dlt;
            ex -= dlt;
            ss = __builtin_ldexp(ss, -2 * dlt);
            zmax = __builtin_ldexp(zmax, -dlt);
            ev1 = rb ? ev2 : ev1;
            ev2 = rb ? it : ev2;
            ev2e = rb ? dlt : ev2e;
        }
        return __builtin_ldexp(pb, ex);
    };
    auto body = [&](const SweepStep<Y>& w, int it, bool last_of_group, bool rescale) {
        const double zv = zvalue(w, it, last_of_group);
        if (store) *zp = zv;
        zp += zstep;
        ss = __fma_rn(zv, zv, ss);
        const bool bigger = fabs(zv) > zmax;
        zmax = fmax(zmax, fabs(zv));
        zmi = bigger ? it : zmi;
        const Y c = mul_add(w.f, b, a);
        a = mul_sub(w.g, a, tau, c);
        b = c;
        if (rescale) {
            const int em = max(y_exp(a), y_exp(b));
            a = y_ldexp(a, -em);
            b = y_ldexp(b, -em);
            ebr += em;
        }
    };
    for (int it0 = 0; it0 < smax; it0 += SW) {
        const int cur = (it0 / SW) & 1;
        const SweepStep<Y> nx = load_sweep_step<Y, DL>(t >> 5, it0 + SW + (t & 31), D, LL, E, P, Pe, Q, Qe, n);
        // a window that holds some lane's twist row runs the second form
        // below for every lane (each step taken only up to the lane's twist
        // row), so that the wave does not run both forms one after the other
        const bool twin = __any(it0 < nsteps && it0 + SW >= nsteps);
        if (!twin && it0 + SW < nsteps) {
            // the twist row lies beyond this window: straight-line steps
            for (int u = 0; u < SW; u += 4) {
                SweepStep<Y> w[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) w[v] = get_sweep_step<Y>(win, cur, side, u + v);
#pragma unroll
                for (int v = 0; v < 4; ++v) body(w[v], it0 + u + v, v == 3, v == 3 && (u & 4));
            }
        } else if (twin && it0 < nsteps) {
            // the same groups of four, each step taken only up to the twist
            // row (step nsteps - 1), which gives z_r; in a short node nearly
            // every window holds some lane's twist row
            const int last = nsteps - 1 - it0;  // step of the twist row
            for (int u = 0; u < SW; u += 4) {
                if (u > last) break;
                SweepStep<Y> w[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) w[v] = get_sweep_step<Y>(win, cur, side, u + v);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int it = it0 + u + v;
                    if (it + 1 < nsteps) body(w[v], it, v == 3, v == 3 && (u & 4));
                    else if (it + 1 == nsteps) h.zr = zvalue(w[v], it, true);
                }
            }
        }
        put_sweep_step<Y>(win, cur ^ 1, t >> 5, t & 31, nx);
        wave_sync();
    }
    h.sp = div(a, b);  // s_r = a_r / b_r  or  p_r = alpha_r / beta_r
    // steps to rows: step s is row s (top) or n-1-s (bottom)
    auto row = [&](int s) -> int64_t { return top ? (int64_t)s : n - 1 - (int64_t)s; };
    h.ss = ss;
    h.zmax = zmax;
    h.zmaxk = zmi < 0 ? -1 : row(zmi);
    h.ev1 = row(ev1);
    h.ev2 = row(ev2);
    h.ev2f = __builtin_ldexp(1.0, -ev2e);
    return h;
}

// (two waves per SIMD: the binary64 instance would otherwise take more than
// half the register file and run alone on its SIMD)
// (DL: nodes without a stored lld, formed from e and d in the sweeps)
template <class Y, int NW, bool DL>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2)))
k_rqi(const ChunkInfo* __restrict__ chunks, int64_t nchunks, const int64_t* __restrict__ list,
      const int64_t* __restrict__ tile_off, int64_t tile_base, double* __restrict__ tiles,
      const Slot* __restrict__ slots, const Node* __restrict__ nodes,
      const Block* __restrict__ blocks, const Y* __restrict__ rep_d, const Y* __restrict__ rep_lld,
      const Y* __restrict__ rep_e, const double* __restrict__ d64, const double* __restrict__ lld64, const Y* __restrict__ P,
      const int* __restrict__ Pe, const Y* __restrict__ Q, const int* __restrict__ Qe,
      const double* __restrict__ P64, const double* __restrict__ Q64, Params prm,
      double eps_y, RqiResult* __restrict__ res, unsigned long long* __restrict__ counters,
      double* __restrict__ work) {
    __shared__ SweepWin<Y> wins[NW];
    __shared__ TwistWin twins[NW];
    const int wv = NW == 1 ? 0 : (int)(threadIdx.x >> 6);
    const int64_t cidx = (int64_t)blockIdx.x * NW + wv;
    if (cidx >= nchunks) return;  // the whole wave: no workgroup barrier follows
    SweepWin<Y>& win = wins[wv];
    TwistWin& twin = twins[wv];
    const int lane = threadIdx.x & 63;
    const int pair = lane >> 1;
    const bool top = (lane & 1) == 0;
    const ChunkInfo ck = chunks[cidx];
    const int64_t idx = ck.begin + pair;
    const bool active = pair < ck.count;
    // tiles of this launch's chunks start at tile_off[0] - tile_base = 0 of
    // `tiles` (one round of a level whose tiles take several)
    double* tile = tiles + (tile_off[cidx] - tile_base) + pair;
    // every pair of the chunk belongs to the same node
    const Node nd = nodes[slots[list[ck.begin]].node];
    const Block bk = blocks[nd.block];
    const int64_t n = bk.n, rep = nd.rep, brow = bk.row0;
    const double spd = nd.spdiam;
    double lo = 0, hi = 0, gap = 0;
    if (active) {
        const Slot sl = slots[list[idx]];
        lo = sl.lo;
        hi = sl.hi;
        double lg = sl.lgap, rg = sl.rgap;
        if (!(lg > 0.0)) lg = (lg < 0.0) ? MR3_BIG : fmax(hi - lo, 1e-300);
        if (!(rg > 0.0)) rg = (rg < 0.0) ? MR3_BIG : fmax(hi - lo, 1e-300);
        gap = fmin(fmin(lg, rg), spd);
    }
    const Y* D = rep_d + rep;
    const Y* LL = rep_lld ? rep_lld + rep : nullptr;
    const Y* E = rep_e + brow;
    const double* D64 = d64 + rep;
    const double* LL64 = lld64 + rep;
    // ---- twist index from a binary64 pass on the copy (argmin |gamma_k|) ----
    const double tau0 = 0.5 * (lo + hi);
    const int64_t hh = n / 2;
    double a = 0, b = 1;
    if (top) { a = -tau0; b = 1.0; } else if (n > 0) { a = D64[n - 1] - tau0; b = 1.0; }
    const int64_t len1 = active ? (top ? hh : n - hh) : 0;
    const int64_t len2 = active ? (top ? n - hh : hh) : 0;
    double gmin = INFINITY;
    int64_t rmin = n / 2;
    prepass_staged(top, D64, LL64, n, tau0, 0, 0, len1, hh, a, b, false, tile, gmin, rmin, twin);
    wave_sync();
    prepass_staged(top, D64, LL64, n, tau0, hh, n - hh, len2, hh, a, b, true, tile, gmin, rmin, twin);
    {
        const double go = __shfl_xor(gmin, 1, 64);
        const int64_t ro = __shfl_xor(rmin, 1, 64);
        if (go < gmin || (go == gmin && ro < rmin)) { gmin = go; rmin = ro; }
    }
    int64_t r = rmin;
    if (r < 0 || r >= n) r = n / 2;
    wave_sync();
    // ---- double-double path: one Rayleigh-quotient step in binary64 on the
    // copy at the midpoint and twist r gives a better starting shift than the
    // midpoint, whose error (the bracket width) costs pairs of small relative
    // gap several double-double sweeps; a result outside the bracket is not
    // used.  (The copy's window space is the double-double window's.) ----
    double lam0 = tau0;
    if (P64 != nullptr) {
        SweepWin<double>& w64 = *reinterpret_cast<SweepWin<double>*>(&win);
        const int64_t st0 = active ? (top ? r + 1 : n - r) : 0;
        Half<double> h0 = sweep_staged<double, false>(top, D64, LL64, nullptr, P64 + brow, Pe + brow, Q64 + brow,
                                               Qe + brow, n, r, tau0, tile, false, st0, w64);
        const double spo = __shfl_xor(h0.sp, 1, 64);
        const double zro = __shfl_xor(h0.zr, 1, 64);
        const double sso = __shfl_xor(h0.ss, 1, 64);
        if (active) {
            const double s_r = top ? h0.sp : spo, p_r = top ? spo : h0.sp;
            const double zrT = top ? h0.zr : zro, zrB = top ? zro : h0.zr;
            const double ssT = top ? h0.ss : sso, ssB = top ? sso : h0.ss;
            const double nrm2 = 1.0 + (r > 0 ? ssT / (zrT * zrT) : 0.0) +
                                (r < n - 1 ? ssB / (zrB * zrB) : 0.0);
            const double l1 = tau0 + ((s_r + p_r) + tau0) / nrm2;
            if (isfinite(l1) && l1 > lo && l1 < hi) lam0 = l1;
        }
        wave_sync();
    }
    // ---- RQI in y at a fixed twist ----
    const double sqn = sqrt((double)(n > 0 ? n : 1));
    const double tol = prm.k_rs * gap * prm.eps_x * sqn;
    Y lam = y_from(lam0, Y());
    bool done = !active;
    bool fallback = prm.force_rqi_fallback != 0;
    int iters = 0;
    Half<Y> mine;
    mine.sp = lam;
    mine.zr = 1.0;
    mine.ss = 0.0;
    mine.zmax = 0.0;
    mine.zmaxk = -1;
    mine.ev1 = top ? 0 : n;
    mine.ev2 = top ? 0 : n;
    mine.ev2f = 1.0;
    Y lam_out = lam;
    double nz2 = 1.0;
    double zT = 1, zB = 1;
    int64_t r_out = r;     // twist of the sweep whose vector is published
    bool retried = false;  // one twist retry after leaving the interval
    // every lane stays in the loop (the staged sweep needs all 64 threads);
    // pairs that are done or falling back sweep zero steps
    for (int it = 0; it < prm.rqi_max_iter; ++it) {
        if (!__any(!done && !fallback)) break;
        const int64_t steps = (done || fallback) ? 0 : (top ? r + 1 : n - r);
        Half<Y> h = sweep_staged<Y, DL>(top, D, LL, E, P + brow, Pe + brow, Q + brow, Qe + brow, n, r,
                                    lam, tile, true, steps, win);
        const Y spo = shfl_y<Y>(h.sp, lane ^ 1);
        const double zro = __shfl_xor(h.zr, 1, 64);
        const double sso = __shfl_xor(h.ss, 1, 64);
        const double rel = h.zmax / fabs(h.zr);
        const double relo = __shfl_xor(rel, 1, 64);
        const int64_t ko = __shfl_xor(h.zmaxk, 1, 64);
        if (done || fallback) continue;
        ++iters;
        const Y s_r = top ? h.sp : spo;
        const Y p_r = top ? spo : h.sp;
        const double zrT = top ? h.zr : zro, zrB = top ? zro : h.zr;
        const double ssT = top ? h.ss : sso, ssB = top ? sso : h.ss;
        const Y gam = add_acc(add_acc(s_r, p_r), lam);
        const double nrm2 = 1.0 + (n > 1 ? ssT / (zrT * zrT) : 0.0) * (r > 0 ? 1.0 : 0.0) +
                            (r < n - 1 ? ssB / (zrB * zrB) : 0.0);
        const double g = to_double(gam);
        if (!(nrm2 >= 1.0) || !isfinite(nrm2) || zrT == 0.0 || zrB == 0.0) {
            fallback = true;
            continue;
        }
        const double resid = fabs(g) / sqrt(nrm2);
        const double corr = g / nrm2;
        const Y lnew = add(lam, y_from(corr, Y()));
        // largest stored entry relative to the twist row, per half (the
        // shuffles above ran on both lanes of every pair, since a shuffle
        // whose source lane is inactive returns 0)
        const double mT = top ? rel : relo;
        const double mB = top ? relo : rel;
        const int64_t kT = top ? h.zmaxk : ko;
        const int64_t kB = top ? ko : h.zmaxk;
        const bool poor_twist = fmax(mT, mB) > 2.0;
        mine = h;
        r_out = r;
        lam_out = lnew;
        nz2 = nrm2;
        zT = zrT;
        zB = zrB;
        if (resid <= tol || fabs(corr) <= 4.0 * eps_y * fabs(hi_of(lam))) {
            done = true;
            continue;
        }
        const double lh = hi_of(lnew);
        if (!(lh >= lo && lh <= hi)) {
            // the Rayleigh quotient left the eigenvalue's interval: with a poor
            // twist the vector was poor, so retry at the same shift with the
            // twist at the largest entry; otherwise fall back to bisection
            if (poor_twist && !retried) {
                retried = true;
                r = (mT >= mB) ? kT : kB;
                continue;
            }
            fallback = true;
            continue;
        }
        lam = lnew;
        // move the twist to the largest entry if the current one is poor
        if (poor_twist) r = (mT >= mB) ? kT : kB;
    }
    // both lanes of a pair agree on `fallback`; a pair that did not converge
    // in rqi_max_iter iterations also falls back
    fallback = active && (fallback || !done);
    if (__any(fallback)) {
        // bisection in y to relative width eps_x sqrt(n) gaptol, then one
        // RQI step (Sec. 2 "Rayleigh quotient iteration"; Sec. 3.2)
        double blo = lo, bhi = hi;
        const int jt = (int)slots[list[active ? idx : 0]].idx;
        // make sure [blo, bhi] brackets eigenvalue jt of the y representation
        bool fixb = fallback;
        for (int it = 0; it < 80; ++it) {
            int c = 0;
            if (fixb) c = negcount_y<Y, DL>(D, LL, E, n, y_from(top ? blo : bhi, Y()));
            const int co = __shfl_xor(c, 1, 64);
            const int clo = top ? c : co, chi = top ? co : c;
            if (fixb) {
                const bool ok = (clo <= jt - 1) && (chi >= jt);
                if (!ok) {
                    const double w = fmax(bhi - blo, fmax(fabs(blo), fabs(bhi)) * 1e-14) + 1e-300;
                    if (clo > jt - 1) blo -= w;
                    if (chi < jt) bhi += w;
                }
                fixb = !ok;
            }
            if (!__any(fixb)) break;
        }
        Y ylo = y_from(blo, Y()), yhi = y_from(bhi, Y());
        const double rt = fmax(prm.eps_x * sqn * prm.gaptol, 8.0 * eps_y);
        bool busy = fallback;
        for (int it = 0; it < 300; ++it) {
            if (busy) {
                const double w = hi_of(sub(yhi, ylo));
                if (!(w > rt * fmax(fabs(hi_of(ylo)), fabs(hi_of(yhi))))) busy = false;
            }
            if (!__any(busy)) break;
            // two interior points: the top lane takes 1/3, the bottom 2/3
            const Y w3 = mul(sub(yhi, ylo), y_from(1.0 / 3.0, Y()));
            const Y x = top ? add(ylo, w3) : add(ylo, add(w3, w3));
            const int j = (int)slots[list[active ? idx : 0]].idx;
            int c = busy ? negcount_y<Y, DL>(D, LL, E, n, x) : 0;
            const int co = __shfl_xor(c, 1, 64);
            const Y xo = shfl_y<Y>(x, lane ^ 1);
            if (busy) {
                const int c1 = top ? c : co, c2 = top ? co : c;
                const Y x1 = top ? x : xo, x2 = top ? xo : x;
                if (c1 >= j) yhi = x1;
                else if (c2 >= j) { ylo = x1; yhi = x2; }
                else ylo = x2;
            }
        }
        lam = mul(add(ylo, yhi), y_from(0.5, Y()));
        // one RQI step at the bisected value; the twist moves to the largest
        // entry of z when the first choice was poor (at most two retries)
        bool again = fallback;
        for (int rep_it = 0; rep_it < 3; ++rep_it) {
            if (!__any(again)) break;
            const int64_t steps = again ? (top ? r + 1 : n - r) : 0;
            Half<Y> h = sweep_staged<Y, DL>(top, D, LL, E, P + brow, Pe + brow, Q + brow, Qe + brow, n, r,
                                        lam, tile, true, steps, win);
            const Y spo = shfl_y<Y>(h.sp, lane ^ 1);
            const double zro = __shfl_xor(h.zr, 1, 64);
            const double sso = __shfl_xor(h.ss, 1, 64);
            const double zmo = __shfl_xor(h.zmax, 1, 64);
            const int64_t zko = __shfl_xor(h.zmaxk, 1, 64);
            if (again) {
                const Y s_r = top ? h.sp : spo;
                const Y p_r = top ? spo : h.sp;
                const double zrT = top ? h.zr : zro, zrB = top ? zro : h.zr;
                const double ssT = top ? h.ss : sso, ssB = top ? sso : h.ss;
                const Y gam = add_acc(add_acc(s_r, p_r), lam);
                const double nrm2 = 1.0 + (r > 0 ? ssT / (zrT * zrT) : 0.0) +
                                    (r < n - 1 ? ssB / (zrB * zrB) : 0.0);
                mine = h;
                r_out = r;
                lam_out = add(lam, y_from(to_double(gam) / nrm2, Y()));
                nz2 = nrm2;
                zT = zrT;
                zB = zrB;
                ++iters;
                const double mT = (top ? h.zmax : zmo) / fabs(zrT);
                const double mB = (top ? zmo : h.zmax) / fabs(zrB);
                const int64_t kT = top ? h.zmaxk : zko, kB = top ? zko : h.zmaxk;
                again = (fmax(mT, mB) > 2.0) && isfinite(nrm2);
                if (again) r = (mT >= mB) ? kT : kB;
            }
        }
    }
    // exchange the per-lane storage bookkeeping and publish the result
    const double zmaxo = __shfl_xor(mine.zmax, 1, 64);
    const int64_t zmaxko = __shfl_xor(mine.zmaxk, 1, 64);
    wave_sync();  // both halves' final stores are visible in the tile
    const int64_t ev1o = __shfl_xor(mine.ev1, 1, 64);
    const int64_t ev2o = __shfl_xor(mine.ev2, 1, 64);
    const double ev2fo = __shfl_xor(mine.ev2f, 1, 64);
    if (active && top) {
        const double nz = sqrt(nz2);
        // sign: largest entry of the final vector positive
        const double cT = (r_out > 0) ? mine.zmax / fabs(zT) : 0.0;
        const double cB = (r_out < n - 1) ? zmaxo / fabs(zB) : 0.0;
        double sgn = 1.0;
        // (the signed largest entry is read back from the tile column)
        if (cT > 1.0 && cT >= cB) sgn = ((tile[mine.zmaxk * 32] < 0) != (zT < 0)) ? -1.0 : 1.0;
        else if (cB > 1.0) sgn = ((tile[zmaxko * 32] < 0) != (zB < 0)) ? -1.0 : 1.0;
        RqiResult o;
        const Y lam_T = add(lam_out, y_from(0.0, Y()));
        o.lam_hi = hi_of(lam_T);
        o.lam_lo = to_double(sub(lam_T, y_from(hi_of(lam_T), Y())));
        o.fT = sgn / (zT * nz);
        o.fB = sgn / (zB * nz);
        o.rowr = sgn / nz;
        o.r = r_out;
        o.evT1 = mine.ev1;
        o.evT2 = mine.ev2;
        o.evT2f = mine.ev2f;
        o.evB1 = ev1o;
        o.evB2 = ev2o;
        o.evB2f = ev2fo;
        o.iters = iters;
        o.status = fallback ? 1 : 0;
        if (!isfinite(o.fT) || !isfinite(o.fB) || !isfinite(o.rowr)) o.status = 2;
        res[idx] = o;
        atomicAdd(&counters[0], (unsigned long long)iters);
        atomicAdd(&work[1], (double)iters * (double)(n + 1));
        atomicAdd(&work[2], (double)n * (P64 != nullptr ? 2.0 : 1.0));  // pre-pass (+ binary64 step)
        if (fallback) atomicAdd(&counters[1], 1ull);
        if (o.status == 2) atomicAdd(&counters[2], 1ull);
    }
}

// ---------------------------------------------------------------------------
// a7: output -- eigenvalue, normalised eigenvector rounded to x, coalesced
// column stores through an LDS transpose (one workgroup per 32 singletons)
// ---------------------------------------------------------------------------
template <class X, class Y>
__global__ void __launch_bounds__(256)
k_zout(const ChunkInfo* __restrict__ chunks, const int64_t* __restrict__ list,
       const int64_t* __restrict__ tile_off, int64_t tile_base, const double* __restrict__ tiles,
       const Slot* __restrict__ slots,
       const Node* __restrict__ nodes, const Block* __restrict__ blocks,
       const ProbInfo* __restrict__ pinfo, const RqiResult* __restrict__ res,
       const ProbDesc* __restrict__ probs, bool any_z) {
    __shared__ double buf[64][33];
    __shared__ int64_t s_n[32], s_r[32], s_col[32], s_evT1[32], s_evT2[32], s_evB1[32], s_evB2[32];
    __shared__ double s_fT[32], s_fB[32], s_rowr[32], s_evT2f[32], s_evB2f[32];
    __shared__ X* s_z[32];
    __shared__ int64_t s_rows;
    const int t = threadIdx.x;
    const ChunkInfo ck = chunks[blockIdx.x];
    const double* tile = tiles + (tile_off[blockIdx.x] - tile_base);
    if (t < 32) {
        const int64_t idx = ck.begin + t;
        s_n[t] = 0;
        if (t < ck.count) {
            const Slot sl = slots[list[idx]];
            const Node nd = nodes[sl.node];
            const Block bk = blocks[nd.block];
            const RqiResult o = res[idx];
            const int p = bk.prob;
            const int sexp = pinfo[p].sexp;
            // eigenvalue of T: lambda[M] + sigma, rounded to x, unscaled
            Y lam = add_acc(mk_y<Y>(o.lam_hi, o.lam_lo), mk_y<Y>(nd.sigma_hi, nd.sigma_lo));
            const ProbDesc pd = probs[p];
            if (blockIdx.y == 0)
                ((__attribute__((address_space(1))) X*)pd.wout)[sl.out] =
                    (X)__builtin_ldexp(to_double(lam), -sexp);
            s_n[t] = bk.n;
            s_r[t] = o.r;
            s_fT[t] = o.fT;
            s_fB[t] = o.fB;
            s_rowr[t] = o.rowr;
            s_evT1[t] = o.evT1;
            s_evT2[t] = o.evT2;
            s_evT2f[t] = o.evT2f;
            s_evB1[t] = o.evB1;
            s_evB2[t] = o.evB2;
            s_evB2f[t] = o.evB2f;
            s_z[t] = pd.zout ? reinterpret_cast<X*>(pd.zout) + sl.out * pd.ldz + bk.start : nullptr;
        }
    }
    __syncthreads();
    if (t == 0) {
        int64_t m = 0;
        for (int q = 0; q < 32; ++q) m = max(m, s_n[q]);
        s_rows = m;
    }
    __syncthreads();
    if (!any_z) return;
    const int64_t rows = s_rows;
    const int wv = t >> 6, ln = t & 63;
    // only the columns of the chunk's pairs are read (a chunk of a small
    // cluster child fills few of its 32); the rows are split over gridDim.y
    // workgroups in blocks of 64
    const int ncol = ck.count;
    const int64_t nblk = (rows + 63) / 64;
    const int64_t bper = (nblk + gridDim.y - 1) / gridDim.y;
    const int64_t rbeg = min<int64_t>(rows, (int64_t)blockIdx.y * bper * 64);
    const int64_t rend = min<int64_t>(rows, rbeg + bper * 64);
    for (int64_t r0 = rbeg; r0 < rend; r0 += 64) {
        for (int e = t; e < 64 * 32; e += 256) {
            const int rr = e >> 5, cc = e & 31;
            if (cc < ncol) buf[rr][cc] = (r0 + rr < rows) ? tile[(r0 + rr) * 32 + cc] : 0.0;
        }
        __syncthreads();
        for (int cc = wv * 8; cc < wv * 8 + 8; ++cc) {
            const int64_t k = r0 + ln;
            if (k >= s_n[cc] || s_z[cc] == nullptr) continue;
            const int64_t r = s_r[cc];
            double v;
            if (k < r) {
                double f = s_fT[cc];
                if (k < s_evT2[cc]) f = (k >= s_evT1[cc]) ? f * s_evT2f[cc] : 0.0;
                v = buf[ln][cc] * f;
            } else if (k == r) {
                v = s_rowr[cc];
            } else {
                double f = s_fB[cc];
                if (k > s_evB2[cc]) f = (k <= s_evB1[cc]) ? f * s_evB2f[cc] : 0.0;
                v = buf[ln][cc] * f;
            }
            // a global store (the pointer came through memory, so the
            // compiler cannot tell its address space; a generic store would
            // also be counted with this workgroup's LDS accesses)
            ((__attribute__((address_space(1))) X*)s_z[cc])[k] = (X)v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// a5: cluster shifts.  k_child_select evaluates 32 candidate shifts on each
// side of a cluster in binary64 on the parent's copy (Sturm count check and
// element growth max |d+_i|); k_child_rep forms the chosen child
// representation in y.
// ---------------------------------------------------------------------------
struct ChildJob {
    int64_t head;     // first slot of the cluster
    int64_t last;     // last slot
    int parent;       // parent node
    int child;        // new node index
    int64_t rep;      // first row of the child representation in the pool
    int64_t tmp;      // first row of the scratch rows
    double tau;       // chosen shift (parent frame), written by k_child_select
    int best;         // 1 if no candidate passed the growth test
    int strict;       // 1 if the growth stayed within k_elg * spdiam
};

__global__ void __launch_bounds__(64)
k_child_select(ChildJob* __restrict__ jobs, int64_t njobs, const Slot* __restrict__ slots,
               const Node* __restrict__ nodes, const Block* __restrict__ blocks,
               const double* __restrict__ d64, const double* __restrict__ lld64, Params prm,
               double ex_over_ey) {
    const int64_t jb = blockIdx.x;
    if (jb >= njobs) return;
    const int lane = threadIdx.x;
    ChildJob job = jobs[jb];
    const Node nd = nodes[job.parent];
    const int64_t n = blocks[nd.block].n;
    const Slot sp = slots[job.head], sq = slots[job.last];
    const double* D = d64 + nd.rep;
    const double* LL = lld64 + nd.rep;
    const bool left = lane < 32;
    const int step = lane & 31;
    const double wid = fmax(sp.hi - sp.lo, sq.hi - sq.lo);
    const double delta0 = fmax(0.25 * wid, 4.0 * 1.1102230246251565e-16 *
                                               fmax(fmax(fabs(sp.lo), fabs(sq.hi)), 1e-300));
    const double delta = __builtin_ldexp(delta0, step);
    const double gapo = left ? sp.lgap : sq.rgap;
    bool valid = !(gapo >= 0.0 && delta > 0.5 * gapo);
    const double tau = left ? sp.lo - delta : sq.hi + delta;
    // stationary transform at tau with element growth max |d+_i| = |c_i / b_i|
    // (approximate reciprocal: the growth only ranks candidates) and inertia;
    // the parent's rows stream through an LDS window filled by the workgroup
    __shared__ double2 win[2][STAGE_ROWS];
    double a = -tau, b = 1.0, gmax = 0.0;
    int negc = 0;
    constexpr int PER = STAGE_ROWS / 64;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = lane + 64 * k;
        if (i < n) win[0][lane + 64 * k] = make_double2(D[i], LL[i]);
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 < n; c0 += STAGE_ROWS) {
        const int cur = (int)((c0 / STAGE_ROWS) & 1);
        double2 nx[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t i = c0 + STAGE_ROWS + lane + 64 * k;
            nx[k] = (i < n) ? make_double2(D[i], LL[i]) : make_double2(0.0, 0.0);
        }
        const int cnt = (int)min<int64_t>(STAGE_ROWS, n - c0);
        auto row = [&](const double2& r, int i) {
            const double c = __fma_rn(r.x, b, a);
            negc += sign_differs(c, b);
            gmax = fmax(gmax, fabs(c) * __builtin_amdgcn_rcp(fabs(b)));
            a = __fma_rn(-tau, c, r.y * a);
            b = c;
            if ((i & 3) == 3) {
                const int em = max(dexp(a), dexp(b));
                a = __builtin_ldexp(a, -em);
                b = __builtin_ldexp(b, -em);
            }
        };
        int i = 0;
        for (; i + 8 <= cnt; i += 8) {
            double2 r[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) r[u] = win[cur][i + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) row(r[u], i + u);
        }
        for (; i < cnt; ++i) row(win[cur][i], i);
#pragma unroll
        for (int k = 0; k < PER; ++k) win[cur ^ 1][lane + 64 * k] = nx[k];
        __syncthreads();
    }
    const int64_t want = left ? sp.idx - 1 : sq.idx;
    // the inertia of the child: from the binary64 copy's count, or, when the
    // cluster ends were refined in y and the outside gap is known, from their
    // brackets (tau lies outside the end bracket and within half the gap to
    // the outside neighbour, whose bracket holds for the representation in y)
    valid = valid && ((prm.refine_ends && gapo >= 0.0) || negc == want) && isfinite(gmax);
    // element growth bound relaxed as the mixed precision analysis allows:
    // k_elg <= max(k_elg, eps_x / (eps_y sqrt(n))) (Sec. 3.2, "Requirements on
    // the representations")
    const double kelg = fmax(prm.k_elg, ex_over_ey / sqrt((double)n));
    const bool pass = valid && !prm.force_best_candidate && gmax <= kelg * nd.spdiam;
    // choose: per side the smallest passing step, then the side with the
    // smaller growth; if nothing passes, the valid candidate of least growth
    const unsigned long long pm = __ballot(pass);
    const unsigned long long vm = __ballot(valid);
    __shared__ double sg[64], st[64];
    sg[lane] = valid ? gmax : INFINITY;
    st[lane] = tau;
    __syncthreads();
    if (lane == 0) {
        int pick = -1, best = 0;
        const unsigned lmask = (unsigned)(pm & 0xffffffffull), rmask = (unsigned)(pm >> 32);
        const int lp = lmask ? __builtin_ctz(lmask) : -1;
        const int rp = rmask ? 32 + __builtin_ctz(rmask) : -1;
        if (lp >= 0 && rp >= 0) pick = (sg[rp] < sg[lp]) ? rp : lp;
        else if (lp >= 0) pick = lp;
        else if (rp >= 0) pick = rp;
        else if (vm) {
            best = 1;
            double g = INFINITY;
            for (int q = 0; q < 64; ++q)
                if (((vm >> q) & 1ull) && sg[q] < g) { g = sg[q]; pick = q; }
        }
        jobs[jb].tau = (pick >= 0) ? st[pick] : sp.lo - delta0;
        jobs[jb].best = (pick >= 0) ? best : 2;
        jobs[jb].strict = (pick >= 0 && !best && sg[pick] <= prm.k_elg * nd.spdiam) ? 1 : 0;
    }
}

template <class Y>
__global__ void __launch_bounds__(64)
k_child_rep(const ChildJob* __restrict__ jobs, int64_t njobs, Slot* __restrict__ slots,
            Node* __restrict__ nodes, const Block* __restrict__ blocks, Y* __restrict__ rep_d,
            Y* __restrict__ rep_lld, const Y* __restrict__ rep_e, double* __restrict__ d64,
            double* __restrict__ lld64, Y* __restrict__ tmpc, int* __restrict__ tmpe, double widen_k,
            double eps_x) {
    const int64_t jb = blockIdx.x;
    if (jb >= njobs) return;
    const int t = threadIdx.x;
    const ChildJob job = jobs[jb];
    const Node pn = nodes[job.parent];
    const Block bk = blocks[pn.block];
    const int64_t n = bk.n;
    const Y* D = rep_d + pn.rep;
    const Y* LL = rep_lld ? rep_lld + pn.rep : nullptr;
    const Y* E = rep_e + bk.row0;
    Y* C = tmpc + job.tmp;
    int* CE = tmpe + job.tmp;
    const Y tau = y_from(job.tau, Y());
    {
        // sequential stationary transform in y by thread 0: c_i = d+_i b_i;
        // the parent's rows stream through an LDS window filled by the
        // workgroup
        __shared__ Y wd[2][STAGE_ROWS], wl[2][STAGE_ROWS];
        constexpr int PER = STAGE_ROWS / 64;
        Y a = neg(tau), b = y_from(1.0, Y());
        int eb = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t i = t + 64 * k;
            if (i < n) {
                wd[0][t + 64 * k] = D[i];
                wl[0][t + 64 * k] = lld_at(LL, E, D, i, n);
            }
        }
        __syncthreads();
        for (int64_t c0 = 0; c0 < n; c0 += STAGE_ROWS) {
            const int cur = (int)((c0 / STAGE_ROWS) & 1);
            Y nd[PER], nl[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int64_t i = c0 + STAGE_ROWS + t + 64 * k;
                nd[k] = (i < n) ? D[i] : y_from(0.0, Y());
                nl[k] = (i < n) ? lld_at(LL, E, D, i, n) : y_from(0.0, Y());
            }
            if (t == 0) {
                const int cnt = (int)min<int64_t>(STAGE_ROWS, n - c0);
                auto row = [&](const Y& dv, const Y& lv, int i) {
                    const Y c = mul_add(dv, b, a);
                    C[c0 + i] = c;
                    CE[c0 + i] = eb;
                    a = mul_sub(lv, a, tau, c);
                    b = c;
                    if ((i & 3) == 3) {
                        const int em = max(y_exp(a), y_exp(b));
                        a = y_ldexp(a, -em);
                        b = y_ldexp(b, -em);
                        eb += em;
                    }
                };
                int i = 0;
                for (; i + 8 <= cnt; i += 8) {  // LDS reads of a block issued first
                    Y dv[8], lv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        dv[u] = wd[cur][i + u];
                        lv[u] = wl[cur][i + u];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) row(dv[u], lv[u], i + u);
                }
                for (; i < cnt; ++i) row(wd[cur][i], wl[cur][i], i);
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                wd[cur ^ 1][t + 64 * k] = nd[k];
                wl[cur ^ 1][t + 64 * k] = nl[k];
            }
            __syncthreads();
        }
    }
    Y* cd = rep_d + job.rep;
    Y* cl = rep_lld ? rep_lld + job.rep : nullptr;
    for (int64_t i = t; i < n; i += blockDim.x) {
        // d+_i = c_i / c_{i-1} (c_{-1} = 1), then lld+_i = e_i^2 / d+_i
        Y dp = C[i];
        if (i > 0) dp = y_ldexp(div(C[i], C[i - 1]), CE[i] - CE[i - 1]);
        cd[i] = dp;
        Y ll = y_from(0.0, Y());
        if (i + 1 < n) ll = div(mul(E[i], E[i]), dp);
        if (cl) cl[i] = ll;
        d64[job.rep + i] = to_double(dp);
        lld64[job.rep + i] = to_double(ll);
    }
    if (t == 0) {
        Node c;
        c.block = pn.block;
        c.depth = pn.depth + 1;
        c.rep = job.rep;
        c.first = job.head;
        c.last = job.last;
        const Y sg = add_acc(mk_y<Y>(pn.sigma_hi, pn.sigma_lo), tau);
        c.sigma_hi = hi_of(sg);
        c.sigma_lo = to_double(sub(sg, y_from(hi_of(sg), Y())));
        c.spdiam = pn.spdiam;
        nodes[job.child] = c;
    }
    // move the cluster's slots to the child; intervals in the child frame,
    // widened by the binary64-copy uncertainty of the parent
    for (int64_t s = job.head + t; s <= job.last; s += blockDim.x) {
        const double lo = slots[s].lo, hi = slots[s].hi;
        const double w = widen_k * (double)n * eps_x * fmax(fabs(lo), fabs(hi));
        slots[s].node = job.child;
        slots[s].lo = (lo - job.tau) - w;
        slots[s].hi = (hi - job.tau) + w;
        slots[s].kind = KIND_NONE;
    }
}

}  // namespace mr3

// Verification of computed eigenpairs (not part of a solve): the accuracy
// measures R and O of the paper's eq. (1).
//   O: Z^T Z - I by FP64 matrix-core tiles (V_MFMA_F64_16X16X4F64); only the
//      upper triangle of 64 x 64 blocks is formed.
//   R: max_i ||T z_i - lambda_i z_i||_1 / ||T||_1, one wave per column.
// The rounding error of the FP64 Gram matrix is bounded by about n * 2^-53
// (inner-product bound), far below the 10 n eps gate it is compared with.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mr3.h"

namespace mr3chk {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// 256 threads = 4 waves; block tile 64 x 64 of G = Z^T Z; each wave owns a
// 32 x 32 quadrant made of 2 x 2 MFMA tiles of 16 x 16; K is staged through
// LDS 16 rows at a time.
__global__ void __launch_bounds__(256)
k_gram(const double* __restrict__ Z, int64_t ldz, int64_t n, int64_t m, double* __restrict__ out) {
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bi > bj) return;  // symmetric: upper triangle of blocks only
    __shared__ double As[16][65];
    __shared__ double Bs[16][65];
    const int t = threadIdx.x;
    const int wv = t >> 6, ln = t & 63;
    const int64_t I0 = bi * 64, J0 = bj * 64;
    const int qi = (wv >> 1) * 32, qj = (wv & 1) * 32;
    v4d acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = 0; k0 < n; k0 += 16) {
        // stage Z[k0..k0+15][I0..I0+63] and Z[k0..k0+15][J0..J0+63]
        for (int e = t; e < 16 * 64; e += 256) {
            const int kk = e & 15, cc = e >> 4;
            const int64_t row = k0 + kk;
            const int64_t ci = I0 + cc, cj = J0 + cc;
            As[kk][cc] = (row < n && ci < m) ? Z[ci * ldz + row] : 0.0;
            Bs[kk][cc] = (row < n && cj < m) ? Z[cj * ldz + row] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 16; ks += 4) {
            // A fragment (16 x 4): lane -> row ln%16 of the tile, k = ln/16
            // B fragment (4 x 16): lane -> k = ln/16, column ln%16
            const int kk = ks + (ln >> 4);
            double af[2], bf[2];
            for (int a = 0; a < 2; ++a) af[a] = As[kk][qi + a * 16 + (ln & 15)];
            for (int b = 0; b < 2; ++b) bf[b] = Bs[kk][qj + b * 16 + (ln & 15)];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // D layout of V_MFMA_F64_16X16X4F64 (checked on the device): register q of
    // lane ln holds row ln/16 + 4q of column ln%16
    double offmax = 0.0, diagmax = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 4; ++q) {
                const int64_t gi = I0 + qi + a * 16 + (ln >> 4) + 4 * q;
                const int64_t gj = J0 + qj + b * 16 + (ln & 15);
                if (gi >= m || gj >= m) continue;
                const double v = acc[a][b][q];
                if (gi == gj) diagmax = fmax(diagmax, fabs(v - 1.0));
                else offmax = fmax(offmax, fabs(v));
            }
    atomic_max_nonneg(&out[0], offmax);
    atomic_max_nonneg(&out[1], diagmax);
}

__global__ void __launch_bounds__(256)
k_tnorm(const double* __restrict__ d, const double* __restrict__ e, int64_t n, double* out) {
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double l = (i > 0) ? fabs(e[i - 1]) : 0.0, r = (i + 1 < n) ? fabs(e[i]) : 0.0;
        v = fmax(v, l + fabs(d[i]) + r);
    }
    atomic_max_nonneg(out, v);
}

// one wave per column
__global__ void __launch_bounds__(256)
k_resid(const double* __restrict__ d, const double* __restrict__ e, const double* __restrict__ W,
        const double* __restrict__ Z, int64_t ldz, int64_t n, int64_t m, double* out) {
    const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int ln = threadIdx.x & 63;
    if (col >= m) return;
    const double* z = Z + col * ldz;
    const double lam = W[col];
    double s = 0.0;
    for (int64_t k = ln; k < n; k += 64) {
        double v = __fma_rn(d[k] - lam, z[k], 0.0);
        if (k > 0) v = __fma_rn(e[k - 1], z[k - 1], v);
        if (k + 1 < n) v = __fma_rn(e[k], z[k + 1], v);
        s += fabs(v);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (ln == 0) atomic_max_nonneg(out, s);
}

}  // namespace mr3chk

extern "C" int mr3_check_f64(mr3_handle h, int64_t n, int64_t m, const double* d, const double* e,
                             const double* W, const double* Z, int64_t ldz, double* orth_out,
                             double* resid_out, void* stream) {
    using namespace mr3chk;
    if (!h) return -1;
    if (n < 0) return -2;
    if (m < 0 || m > n) return -3;
    if (n > 0 && !d) return -4;
    if (n > 1 && !e) return -5;
    if (m > 0 && !W) return -6;
    if (m > 0 && !Z) return -7;
    if (ldz < (n > 1 ? n : 1)) return -8;
    if (!orth_out) return -9;
    if (!resid_out) return -10;
    orth_out[0] = orth_out[1] = 0.0;
    resid_out[0] = 0.0;
    if (n == 0 || m == 0) return MR3_OK;
    hipStream_t st = (hipStream_t)stream;
    double* buf = nullptr;
    if (hipMalloc(&buf, 4 * sizeof(double)) != hipSuccess) return MR3_ERR_HIP;
    hipError_t err = hipMemsetAsync(buf, 0, 4 * sizeof(double), st);
    const unsigned nb = (unsigned)((m + 63) / 64);
    if (err == hipSuccess) {
        hipLaunchKernelGGL(k_gram, dim3(nb, nb), dim3(256), 0, st, Z, ldz, n, m, buf);
        hipLaunchKernelGGL(k_tnorm, dim3(64), dim3(256), 0, st, d, e ? e : d, n, buf + 2);
        hipLaunchKernelGGL(k_resid, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, d, e ? e : d, W,
                           Z, ldz, n, m, buf + 3);
        err = hipGetLastError();
    }
    double hb[4] = {0, 0, 0, 0};
    if (err == hipSuccess) err = hipMemcpyAsync(hb, buf, sizeof(hb), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (err != hipSuccess) return MR3_ERR_HIP;
    orth_out[0] = hb[0];
    orth_out[1] = hb[1];
    resid_out[0] = hb[2] > 0 ? hb[3] / hb[2] : hb[3];
    return MR3_OK;
}

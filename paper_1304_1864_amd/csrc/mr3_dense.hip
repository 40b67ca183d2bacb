// Dense symmetric and Hermitian eigenproblems (Sec. 4.2, Fig. 3): the
// Householder reduction to tridiagonal form A = Q T Q^H and the
// back-transformation Z := Q Z are rocSOLVER's (sytrd/hetrd, ormtr/unmtr);
// the eigenpairs of T come from this library's mixed-precision solver.  The
// reduction dominates the time for large n (O(n^3) against O(kn) for k
// eigenpairs of T), so the pipeline's point is the accuracy the tridiagonal
// stage carries over to A.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>
#include <stdint.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>
#include <unordered_map>

#include "../../include/mr3.h"
#include "mr3_internal.h"

namespace {

// one rocBLAS handle per library handle, made on first use on its device
std::mutex g_mu;
std::unordered_map<mr3_handle, rocblas_handle> g_blas;

rocblas_handle blas_of(mr3_handle h) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_blas.find(h);
    if (it != g_blas.end()) return it->second;
    rocblas_handle bh = nullptr;
    if (rocblas_create_handle(&bh) != rocblas_status_success) return nullptr;
    g_blas[h] = bh;
    return bh;
}

struct DevMem {
    void* p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
    bool alloc(size_t bytes) { return hipMalloc(&p, std::max<size_t>(bytes, 1)) == hipSuccess; }
};

int check_dense(mr3_handle h, int64_t n, const void* A, int64_t lda, int range, double vl,
                double vu, int64_t il, int64_t iu, const int64_t* m, const void* W, const void* Z,
                int64_t ldz) {
    if (!h) return -1;
    if (n < 0 || n > INT_MAX) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max<int64_t>(1, n) || lda > INT_MAX) return -4;
    if (range < MR3_RANGE_ALL || range > MR3_RANGE_INDEX) return -5;
    if (range == MR3_RANGE_VALUE && !(vl < vu)) return -7;
    if (range == MR3_RANGE_INDEX && (il < 1 || iu > n || il > iu + 1)) return il < 1 ? -8 : -9;
    if (!m) return -10;
    if (n > 0 && !W) return -11;
    if (Z && (ldz < std::max<int64_t>(1, n) || ldz > INT_MAX)) return -13;
    return 0;
}

// real eigenvectors of T (n x m, leading dimension n) into the complex Z
// (R2: float2 or double2, real part first)
template <class R, class R2>
__global__ void __launch_bounds__(256)
k_real_to_complex(const R* __restrict__ zr, int64_t n, int64_t m, R2* __restrict__ z, int64_t ldz) {
    const int64_t total = n * m;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / n, i = t - j * n;
        R2 v;
        v.x = zr[t];
        v.y = R(0);
        z[j * ldz + i] = v;
    }
}

template <class X>
struct Real;
template <>
struct Real<float> {
    static rocblas_status trd(rocblas_handle b, rocblas_int n, float* A, rocblas_int lda, float* D,
                              float* E, float* tau) {
        return rocsolver_ssytrd(b, rocblas_fill_lower, n, A, lda, D, E, tau);
    }
    static rocblas_status mtr(rocblas_handle b, rocblas_int n, rocblas_int m, float* A,
                              rocblas_int lda, float* tau, float* Z, rocblas_int ldz) {
        return rocsolver_sormtr(b, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, n,
                                m, A, lda, tau, Z, ldz);
    }
    static int solve(mr3_handle h, int64_t n, const float* d, const float* e, int range, double vl,
                     double vu, int64_t il, int64_t iu, int64_t* m, float* W, float* Z,
                     int64_t ldz, void* stream) {
        return mr3_solve_f32(h, n, d, e, range, vl, vu, il, iu, m, W, Z, ldz, nullptr, 0, stream);
    }
};
template <>
struct Real<double> {
    static rocblas_status trd(rocblas_handle b, rocblas_int n, double* A, rocblas_int lda,
                              double* D, double* E, double* tau) {
        return rocsolver_dsytrd(b, rocblas_fill_lower, n, A, lda, D, E, tau);
    }
    static rocblas_status mtr(rocblas_handle b, rocblas_int n, rocblas_int m, double* A,
                              rocblas_int lda, double* tau, double* Z, rocblas_int ldz) {
        return rocsolver_dormtr(b, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, n,
                                m, A, lda, tau, Z, ldz);
    }
    static int solve(mr3_handle h, int64_t n, const double* d, const double* e, int range,
                     double vl, double vu, int64_t il, int64_t iu, int64_t* m, double* W,
                     double* Z, int64_t ldz, void* stream) {
        return mr3_solve_f64(h, n, d, e, range, vl, vu, il, iu, m, W, Z, ldz, nullptr, 0, stream);
    }
};

// the work of a call has ended on its stream before its buffers are freed
int finish(int rc, hipStream_t st) {
    if (hipStreamSynchronize(st) != hipSuccess && rc == MR3_OK) rc = MR3_ERR_HIP;
    return rc;
}

template <class X>
int dense_real(mr3_handle h, int64_t n, X* A, int64_t lda, int range, double vl, double vu,
               int64_t il, int64_t iu, int64_t* m, X* W, X* Z, int64_t ldz, void* stream) {
    int rc = check_dense(h, n, A, lda, range, vl, vu, il, iu, m, W, Z, ldz);
    if (rc) return rc;
    *m = 0;
    if (n == 0 || (range == MR3_RANGE_INDEX && il > iu)) return MR3_OK;
    const hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(mr3_handle_device(h)) != hipSuccess) return MR3_ERR_HIP;
    rocblas_handle bh = blas_of(h);
    if (!bh || rocblas_set_stream(bh, st) != rocblas_status_success) return MR3_ERR_HIP;
    DevMem mem;  // d, e and the reflector scalars
    if (!mem.alloc(3 * (size_t)n * sizeof(X))) return MR3_ERR_HIP;
    X* D = (X*)mem.p;
    X* E = D + n;
    X* tau = E + n;
    if (Real<X>::trd(bh, (rocblas_int)n, A, (rocblas_int)lda, D, E, tau) != rocblas_status_success)
        return finish(MR3_ERR_HIP, st);
    rc = Real<X>::solve(h, n, D, E, range, vl, vu, il, iu, m, W, Z, ldz, stream);
    if (rc == MR3_OK && Z && *m > 0 &&
        Real<X>::mtr(bh, (rocblas_int)n, (rocblas_int)*m, A, (rocblas_int)lda, tau, Z,
                     (rocblas_int)ldz) != rocblas_status_success)
        rc = MR3_ERR_HIP;
    return finish(rc, st);
}

template <class R>
struct Cplx;
template <>
struct Cplx<float> {
    using C = rocblas_float_complex;
    using R2 = float2;
    static rocblas_status trd(rocblas_handle b, rocblas_int n, C* A, rocblas_int lda, float* D,
                              float* E, C* tau) {
        return rocsolver_chetrd(b, rocblas_fill_lower, n, A, lda, D, E, tau);
    }
    static rocblas_status mtr(rocblas_handle b, rocblas_int n, rocblas_int m, C* A,
                              rocblas_int lda, C* tau, C* Z, rocblas_int ldz) {
        return rocsolver_cunmtr(b, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, n,
                                m, A, lda, tau, Z, ldz);
    }
};
template <>
struct Cplx<double> {
    using C = rocblas_double_complex;
    using R2 = double2;
    static rocblas_status trd(rocblas_handle b, rocblas_int n, C* A, rocblas_int lda, double* D,
                              double* E, C* tau) {
        return rocsolver_zhetrd(b, rocblas_fill_lower, n, A, lda, D, E, tau);
    }
    static rocblas_status mtr(rocblas_handle b, rocblas_int n, rocblas_int m, C* A,
                              rocblas_int lda, C* tau, C* Z, rocblas_int ldz) {
        return rocsolver_zunmtr(b, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, n,
                                m, A, lda, tau, Z, ldz);
    }
};

// Hermitian A: the reduction leaves a real tridiagonal, solved by the real
// solver of the same precision; its real eigenvectors are widened to complex
// before the back-transformation
template <class R>
int dense_complex(mr3_handle h, int64_t n, void* A, int64_t lda, int range, double vl, double vu,
                  int64_t il, int64_t iu, int64_t* m, R* W, void* Z, int64_t ldz, void* stream) {
    using C = typename Cplx<R>::C;
    int rc = check_dense(h, n, A, lda, range, vl, vu, il, iu, m, W, Z, ldz);
    if (rc) return rc;
    *m = 0;
    if (n == 0 || (range == MR3_RANGE_INDEX && il > iu)) return MR3_OK;
    const hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(mr3_handle_device(h)) != hipSuccess) return MR3_ERR_HIP;
    rocblas_handle bh = blas_of(h);
    if (!bh || rocblas_set_stream(bh, st) != rocblas_status_success) return MR3_ERR_HIP;
    auto* Ac = (C*)A;
    // d, e (real) and the complex reflector scalars; the real eigenvectors of
    // T (at most n columns: the count of a value range is not known before)
    const int64_t kcap = range == MR3_RANGE_INDEX ? iu - il + 1 : n;
    if (Z && (size_t)kcap > SIZE_MAX / sizeof(R) / (size_t)n) return -2;  // n kcap reals
    DevMem mem, zr;
    if (!mem.alloc(2 * (size_t)n * sizeof(R) + (size_t)n * sizeof(C))) return MR3_ERR_HIP;
    if (Z && !zr.alloc((size_t)n * (size_t)kcap * sizeof(R))) return MR3_ERR_HIP;
    auto* tau = (C*)mem.p;  // (the complex scalars first: their alignment)
    R* D = (R*)(tau + n);
    R* E = D + n;
    if (Cplx<R>::trd(bh, (rocblas_int)n, Ac, (rocblas_int)lda, D, E, tau) != rocblas_status_success)
        return finish(MR3_ERR_HIP, st);
    rc = Real<R>::solve(h, n, D, E, range, vl, vu, il, iu, m, W, Z ? (R*)zr.p : nullptr, n, stream);
    if (rc == MR3_OK && Z && *m > 0) {
        const int64_t total = n * *m;
        const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
        hipLaunchKernelGGL((k_real_to_complex<R, typename Cplx<R>::R2>), dim3(grid), dim3(256), 0,
                           st, (const R*)zr.p, n, *m, (typename Cplx<R>::R2*)Z, ldz);
        if (hipGetLastError() != hipSuccess ||
            Cplx<R>::mtr(bh, (rocblas_int)n, (rocblas_int)*m, Ac, (rocblas_int)lda, tau, (C*)Z,
                         (rocblas_int)ldz) != rocblas_status_success)
            rc = MR3_ERR_HIP;
    }
    return finish(rc, st);
}

}  // namespace

void mr3_dense_release(mr3_handle h) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_blas.find(h);
    if (it == g_blas.end()) return;
    (void)rocblas_destroy_handle(it->second);
    g_blas.erase(it);
}

extern "C" {

int mr3_dense_f32(mr3_handle h, int64_t n, float* A, int64_t lda, int range, double vl,
                  double vu, int64_t il, int64_t iu, int64_t* m, float* W, float* Z, int64_t ldz,
                  void* stream) {
    return dense_real<float>(h, n, A, lda, range, vl, vu, il, iu, m, W, Z, ldz, stream);
}

int mr3_dense_f64(mr3_handle h, int64_t n, double* A, int64_t lda, int range, double vl,
                  double vu, int64_t il, int64_t iu, int64_t* m, double* W, double* Z,
                  int64_t ldz, void* stream) {
    return dense_real<double>(h, n, A, lda, range, vl, vu, il, iu, m, W, Z, ldz, stream);
}

int mr3_dense_c64(mr3_handle h, int64_t n, void* A, int64_t lda, int range, double vl,
                  double vu, int64_t il, int64_t iu, int64_t* m, float* W, void* Z, int64_t ldz,
                  void* stream) {
    return dense_complex<float>(h, n, A, lda, range, vl, vu, il, iu, m, W, Z, ldz, stream);
}

int mr3_dense_c128(mr3_handle h, int64_t n, void* A, int64_t lda, int range, double vl,
                   double vu, int64_t il, int64_t iu, int64_t* m, double* W, void* Z, int64_t ldz,
                   void* stream) {
    return dense_complex<double>(h, n, A, lda, range, vl, vu, il, iu, m, W, Z, ldz, stream);
}

}  // extern "C"

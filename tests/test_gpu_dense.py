"""Parity of the dense pipeline (Sec. 4.2, Fig. 3: A = Q T Q^H reduced to
tridiagonal form, this library's solver, back-transformation) with the
oracle, through the C ABI.

Inputs are the paper's dense kind (random orthogonal / unitary similarity
transforms of the tridiagonal test matrices, whose eigenvalues the
tridiagonal oracle gives directly) and random symmetric matrices (eigenvalues
from the dense oracle's own Householder reduction).  Gates: eigenvalues
within 4 n eps ||A||_1 of the oracle's (plus the rounding of A itself),
residual max_i ||A z_i - lambda_i z_i||_1 / ||A||_1 and orthogonality
max |Z^H Z - I| within 10 n eps."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import dense as OD

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr3():
    import paper_1304_1864_amd as lib

    lib.load_library()
    return lib


def _norm1(A):
    return float(np.abs(A).sum(axis=0).max())


def check(mr3, A, ref, eps, il=1, iu=None, rng="all"):
    n = A.shape[0]
    print(f"dense case n={n} dtype={A.dtype} range={rng} il={il} iu={iu}", flush=True)
    Ag = torch.from_numpy(np.ascontiguousarray(A)).to("cuda:0")
    Wg, Zg = mr3.dense(Ag, range=rng, il=il, iu=iu)
    torch.cuda.synchronize()
    # the input is not modified (the binding reduces a column-major copy)
    assert torch.equal(Ag.cpu(), torch.from_numpy(np.ascontiguousarray(A)))
    w = Wg.double().cpu().numpy()
    Z = Zg.cpu().numpy().astype(np.complex128 if np.iscomplexobj(A) else np.float64)
    A64 = A.astype(np.complex128 if np.iscomplexobj(A) else np.float64)
    nA = _norm1(A64)
    assert w.size == ref.size
    assert np.all(np.diff(w) >= 0)
    err = np.abs(w - ref).max() / (n * eps * nA)
    R = np.abs(A64 @ Z - Z * w[None, :]).sum(axis=0).max() / (nA * n * eps)
    O = np.abs(Z.conj().T @ Z - np.eye(w.size)).max() / (n * eps)
    print(f"    eig {err:.3g}  R {R:.3g}  O {O:.3g}  (units of n eps)", flush=True)
    assert err <= 4.0 + 2.0, err
    assert R <= 10.0, R
    assert O <= 10.0, O
    return err, R, O


@pytest.mark.parametrize("n", [1, 2, 37, 600])
def test_dense_qtq_f64(mr3, n):
    d, e, _ = W.prescribed_spectrum(n, 11)
    A = W.dense_from_tridiagonal(d, e, 12)
    hi, lo = oracle.eigvals(d, e)
    check(mr3, A, hi + lo, 2.0 ** -53)


def test_dense_normal_f64_against_dense_oracle(mr3):
    A = W.dense_normal(500, 13)
    hi, lo = OD.eigvals(A)
    check(mr3, A, hi + lo, 2.0 ** -53)


def test_dense_subset_f64(mr3):
    d, e, _ = W.prescribed_spectrum(400, 14)
    A = W.dense_from_tridiagonal(d, e, 15)
    hi, lo = oracle.eigvals(d, e, 20, 90)
    check(mr3, A, hi + lo, 2.0 ** -53, il=20, iu=90, rng="index")


def test_dense_qtq_f32(mr3):
    d, e = W.uniform(500, 16, np.float64)
    A = W.dense_from_tridiagonal(d, e, 17, dtype=np.float32)
    hi, lo = OD.eigvals(A.astype(np.float64))
    check(mr3, A, hi + lo, 2.0 ** -24)


@pytest.mark.parametrize("n", [3, 300])
def test_dense_hermitian_c128(mr3, n):
    d, e, _ = W.prescribed_spectrum(n, 18)
    A = W.dense_from_tridiagonal(d, e, 19, complex_=True)
    hi, lo = oracle.eigvals(d, e)
    check(mr3, A, hi + lo, 2.0 ** -53)


def test_dense_hermitian_c64(mr3):
    """Single-complex Hermitian input: eigenvalues against the dense oracle of
    the rounded matrix, vectors at the FP32 gates."""
    d, e = W.uniform(200, 20, np.float64)
    A = W.dense_from_tridiagonal(d, e, 21, complex_=True).astype(np.complex64)
    hi, lo = OD.eigvals(A.astype(np.complex128))
    check(mr3, A, hi + lo, 2.0 ** -24)


def test_dense_argument_errors(mr3):
    lib = mr3.load_library()
    h = mr3.default_handle()
    A = torch.zeros((4, 4), dtype=torch.float64, device="cuda:0")
    W_ = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    m = ctypes.c_int64(0)
    p = ctypes.c_void_p
    assert lib.mr3_dense_f64(None, 4, p(A.data_ptr()), 4, 0, 0.0, 0.0, 1, 4, ctypes.byref(m),
                             p(W_.data_ptr()), None, 4, None) == -1
    assert lib.mr3_dense_f64(h.ptr, 4, p(A.data_ptr()), 3, 0, 0.0, 0.0, 1, 4, ctypes.byref(m),
                             p(W_.data_ptr()), None, 4, None) == -4
    assert lib.mr3_dense_f64(h.ptr, 1 << 31, p(A.data_ptr()), 1 << 31, 0, 0.0, 0.0, 1, 4,
                             ctypes.byref(m), p(W_.data_ptr()), None, 4, None) == -2
    assert lib.mr3_dense_c128(h.ptr, 4, p(A.data_ptr()), 4, 2, 0.0, 0.0, 0, 4, ctypes.byref(m),
                              p(W_.data_ptr()), None, 4, None) == -8
    assert lib.mr3_dense_f64(h.ptr, 0, None, 1, 0, 0.0, 0.0, 1, 0, ctypes.byref(m), None, None, 1,
                             None) == 0 and m.value == 0

"""Parity of the HIP path with the CPU oracle (needs an MI355X).

Every case calls the library through its C ABI (the ctypes binding), compares
eigenvalues with the oracle's double-double values and eigenvectors through
residual, orthogonality and per-group subspace angles against the gates in
tests/metrics.py.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests import metrics as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr3():
    import paper_1304_1864_amd as lib

    lib.load_library()
    return lib


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def run_case(mr3, d, e, rng="all", il=1, iu=None, vl=0.0, vu=0.0, vectors=True, check_angles=True,
             oracle_w=None, handle=None):
    n = d.size
    eps = M.eps_of(d.dtype)
    print(f"case n={n} dtype={d.dtype} range={rng} il={il} iu={iu}", flush=True)
    Wg, Zg = mr3.solve(_dev(d), _dev(e), range=rng, il=il, iu=iu, vl=vl, vu=vu, vectors=vectors,
                       handle=handle)
    torch.cuda.synchronize()
    w = Wg.double().cpu().numpy()
    d64, e64 = d.astype(np.float64), e.astype(np.float64)
    tn = M.tnorm(d64, e64)
    if rng == "value":
        il = oracle.count(d64, e64, vl) + 1
        iu = oracle.count(d64, e64, vu)
    if rng == "all":
        il, iu = 1, n
    if iu is None:
        iu = n
    assert w.size == max(iu - il + 1, 0), (w.size, il, iu)
    if w.size == 0:
        return {}
    if oracle_w is None:
        hi, lo = oracle.eigvals(d64, e64, il, iu)
    else:
        hi, lo = oracle_w
    ref = hi + lo
    err = float(np.max(np.abs(w - ref)))
    assert np.all(np.diff(w) >= 0), "eigenvalues not ascending"
    assert err <= 4 * n * eps * tn, f"eigenvalue error {err:.3e} > {4 * n * eps * tn:.3e}"
    out = {"eig_err": err / (n * eps * tn)}
    if vectors:
        Z = Zg.double().cpu().numpy()
        R = M.residual(d64, e64, w, Z)
        O = M.orthogonality(Z)
        assert R <= 10 * n * eps, f"residual {R:.3e}"
        assert O <= 10 * n * eps, f"orthogonality {O:.3e}"
        out.update(R=R / (n * eps), O=O / (n * eps))
        if check_angles:
            Zr = oracle.eigvecs(d64, e64, hi, lo)
            ratio, worst = M.subspace_sines(ref, Zr, Z, R, tn, group_tol=1e-8 * tn)
            assert ratio <= 1.0, f"subspace angle {worst:.3e} above its bound (ratio {ratio:.2f})"
            out.update(sin=worst)
    print("   ", {k: f"{v:.3g}" for k, v in out.items()}, flush=True)
    return out


def test_121_f32_closed_form(mr3):
    for n in (1, 2, 3, 64, 512):
        d, e = W.toeplitz_121(n, np.float32)
        Wg, Zg = mr3.solve(_dev(d), _dev(e))
        w = Wg.double().cpu().numpy()
        assert np.max(np.abs(w - W.toeplitz_121_eigs(n))) <= 4 * n * 2.0 ** -24 * 4
        Z = Zg.double().cpu().numpy()
        j = np.arange(1, n + 1)
        for i in range(n):
            v = np.sqrt(2.0 / (n + 1)) * np.sin(j * (n - i) * np.pi / (n + 1))
            c = abs(v @ Z[:, i])
            assert 1 - c <= 1e-4, (n, i, c)
        run_case(mr3, d, e)


def test_uniform_f32_512(mr3):
    d, e = W.uniform(512, 0, np.float32)
    run_case(mr3, d, e)


def test_uniform_f64_small(mr3):
    for n, seed in ((5, 1), (37, 2), (200, 3)):
        d, e = W.uniform(n, seed, np.float64)
        run_case(mr3, d, e)


def test_glued_wilkinson_f64_336(mr3):
    d, e = W.glued_wilkinson(336)
    run_case(mr3, d, e)


def test_prescribed_f64(mr3):
    d, e, _ = W.prescribed_spectrum(600, 1)
    run_case(mr3, d, e)
    run_case(mr3, d, e, rng="index", il=1, iu=60)
    run_case(mr3, d, e, rng="index", il=250, iu=320)


def test_clement(mr3):
    for dt in (np.float32, np.float64):
        d, e = W.clement(101, dt)
        run_case(mr3, d, e)


def test_value_range(mr3):
    d, e = W.uniform(300, 9, np.float64)
    run_case(mr3, d, e, rng="value", vl=-0.5, vu=0.25)
    d, e = W.uniform(300, 9, np.float32)
    run_case(mr3, d, e, rng="value", vl=-0.5, vu=0.25)


def test_split_blocks(mr3):
    # three blocks: zero couplings split the matrix
    d, e = W.uniform(90, 4, np.float64)
    e[29] = 0.0
    e[59] = 1e-300
    run_case(mr3, d, e)
    run_case(mr3, d, e, rng="index", il=10, iu=70)
    run_case(mr3, d, e, rng="value", vl=-0.3, vu=0.6)


def test_edge_sizes(mr3):
    for n in (0, 1, 2):
        for dt in (np.float32, np.float64):
            d, e = W.uniform(max(n, 1), 5, dt)
            d, e = d[:n], e[: max(n - 1, 0)]
            if n == 0:
                Wg, Zg = mr3.solve(_dev(d), _dev(e))
                assert Wg.numel() == 0 and Zg.shape[1] == 0
                continue
            run_case(mr3, d, e)

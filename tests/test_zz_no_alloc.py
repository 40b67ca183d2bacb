"""mr3_solve_noalloc (needs an MI355X): the solve that allocates nothing runs
on the library's static scratch array and gives the results of the ordinary
entry points (mr3_solve_f32 / mr3_solve_f64 on the handle's pool) to the
gates: eigenvalues within 4 n eps ||T||_1 of each other and of the oracle,
residual and orthogonality within 10 n eps, eigenvectors within the
alone-vs-mix criteria.  Two calls in a row on one GPU, the second smaller,
so the second runs on what the first left in the scratch."""
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


def _compare(mr3, h, d, e, rng="all", il=1, iu=None):
    n = d.size
    eps = M.eps_of(d.dtype)
    print(f"noalloc n={n} {np.dtype(d.dtype).name} range={rng}", flush=True)
    Wn, Zn = mr3.solve(_dev(d), _dev(e), range=rng, il=il, iu=iu, handle=h, noalloc=True)
    Wp, Zp = mr3.solve(_dev(d), _dev(e), range=rng, il=il, iu=iu, handle=h)
    d64, e64 = d.astype(np.float64), e.astype(np.float64)
    tn = M.tnorm(d64, e64)
    if iu is None:
        iu = n
    wn, wp = Wn.double().cpu().numpy(), Wp.double().cpu().numpy()
    assert wn.size == wp.size == iu - il + 1
    hi, lo = oracle.eigvals(d64, e64, il, iu)
    assert np.max(np.abs(wn - (hi + lo))) <= 4 * n * eps * tn
    Zn_, Zp_ = Zn.double().cpu().numpy(), Zp.double().cpu().numpy()
    Rn, On = M.residual(d64, e64, wn, Zn_), M.orthogonality(Zn_)
    Rp, Op = M.residual(d64, e64, wp, Zp_), M.orthogonality(Zp_)
    assert Rn <= 10 * n * eps and On <= 10 * n * eps
    c, g, ng = M.alone_vs_mix(wp, Zp_, wn, Zn_, max(Rn, Rp), max(On, Op), tn, eps)
    print(f"   R {Rn / (n * eps):.3g} n eps, O {On / (n * eps):.3g} n eps; vs pool 1-|cos| {c:.3g}, "
          f"groups {ng} sin/bound {g:.3g}", flush=True)


def test_noalloc_matches_the_pool_solves(mr3):
    h = mr3.Handle(0)
    # first call: a problem whose tiles exceed the scratch (rounds) and whose
    # tree has clusters; second call: a smaller one on the same scratch
    d, e, _ = W.prescribed_spectrum(3000, 6)
    _compare(mr3, h, d, e)
    d, e = W.glued_wilkinson(1000)
    _compare(mr3, h, d, e, rng="index", il=100, iu=700)
    d, e = W.toeplitz_121_noisy(2500, 7, 1e-6, np.float32)
    _compare(mr3, h, d, e)
    d, e = W.uniform(400, 8, np.float32)
    _compare(mr3, h, d, e)


def test_noalloc_refuses_sizes_beyond_the_maximum(mr3):
    h = mr3.Handle(0)
    n = mr3.MR3_NOALLOC_MAX_N + 1
    d = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(mr3.MR3Error) as ei:
        mr3.solve(d, d[: n - 1], handle=h, noalloc=True)
    assert ei.value.code == -3

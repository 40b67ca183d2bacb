"""Solves on a caller's work region (needs an MI355X): the query's size runs
the same launches as the handle's pool (bitwise-equal results); the minimum
size walks the representation tree one cluster per group and computes the
eigenvectors in rounds of one chunk, and still meets every gate against the
oracle; a region below the minimum is refused with the position of
work_bytes."""
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


def _region(nbytes):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda:0")


CASES = {
    "uniform-fp32-1000": lambda: W.uniform(1000, 3, np.float32),
    "prescribed-fp64-2000": lambda: W.prescribed_spectrum(2000, 4)[:2],
    "glued-fp64-1344": lambda: W.glued_wilkinson(1344),
}


@pytest.mark.parametrize("case", list(CASES))
def test_query_size_matches_pool(mr3, case):
    d, e = CASES[case]()
    n = d.size
    prec = 32 if d.dtype == np.float32 else 64
    h = mr3.Handle(0)
    q = mr3.mr3_workspace_bytes(h, n, mr3.RANGE_ALL, 0, prec)
    print(f"{case}: query {q / 2 ** 20:.1f} MiB", flush=True)
    W0, Z0 = mr3.solve(_dev(d), _dev(e), handle=h)
    W1, Z1 = mr3.solve(_dev(d), _dev(e), handle=h, work=_region(q))
    assert torch.equal(W0, W1) and torch.equal(Z0, Z1)


@pytest.mark.parametrize("case", list(CASES))
def test_minimum_size_meets_the_gates(mr3, case):
    """Depth-first groups of one cluster and one-chunk eigenvector rounds:
    every gate against the oracle, and the same results as the pool solve to
    the alone-vs-mix criteria (the child multisection shape depends on the
    group, so the bits may differ)."""
    d, e = CASES[case]()
    n = d.size
    prec = 32 if d.dtype == np.float32 else 64
    eps = M.eps_of(d.dtype)
    h = mr3.Handle(0)
    low = mr3.mr3_workspace_min_bytes(h, n, mr3.RANGE_ALL, 0, prec)
    print(f"{case}: minimum {low / 2 ** 20:.1f} MiB", flush=True)
    W0, Z0 = mr3.solve(_dev(d), _dev(e), handle=h)
    W1, Z1 = mr3.solve(_dev(d), _dev(e), handle=h, work=_region(low))
    st = h.stats()
    d64, e64 = d.astype(np.float64), e.astype(np.float64)
    tn = M.tnorm(d64, e64)
    w1 = W1.double().cpu().numpy()
    hi, lo = oracle.eigvals(d64, e64)
    assert np.max(np.abs(w1 - (hi + lo))) <= 4 * n * eps * tn
    Z1n = Z1.double().cpu().numpy()
    R1, O1 = M.residual(d64, e64, w1, Z1n), M.orthogonality(Z1n)
    assert R1 <= 10 * n * eps and O1 <= 10 * n * eps
    Zr = oracle.eigvecs(d64, e64, hi, lo)
    ratio, worst = M.subspace_sines(hi + lo, Zr, Z1n, R1, tn, 1e-8 * tn, O=O1)
    assert ratio <= 1.0
    Z0n = Z0.double().cpu().numpy()
    R0, O0 = M.residual(d64, e64, W0.double().cpu().numpy(), Z0n), M.orthogonality(Z0n)
    c, g, ng = M.alone_vs_mix(W0.double().cpu().numpy(), Z0n, w1, Z1n, max(R0, R1), max(O0, O1), tn, eps)
    print(f"   clusters {st['n_clusters']} d_max {st['d_max']}; vs pool: 1-|cos| {c:.3g}, "
          f"groups {ng}, sin/bound {g:.3g}", flush=True)


def test_too_small_and_batched(mr3):
    d, e, _ = W.prescribed_spectrum(700, 5)
    h = mr3.Handle(0)
    low = mr3.mr3_workspace_min_bytes(h, d.size, mr3.RANGE_ALL, 0, 64)
    with pytest.raises(mr3.MR3Error) as ei:
        mr3.solve(_dev(d), _dev(e), handle=h, work=_region(low // 4))
    assert ei.value.code == -15
    probs = W.batch_normal(48, 32, 300, seed=9, dtype=np.float64)
    probs[5] = W.glued_wilkinson(105)
    sizes = [p[0].size for p in probs]
    ds, es = [_dev(p[0]) for p in probs], [_dev(p[1]) for p in probs]
    with pytest.raises(mr3.MR3Error) as ei:
        mr3.solve_batched(ds, es, handle=h, work=_region(4096))
    assert ei.value.code == -16
    q = mr3.mr3_workspace_bytes_batched(h, 64, sizes)
    Wa, Za = mr3.solve_batched(ds, es, handle=h)
    Wb, Zb = mr3.solve_batched(ds, es, handle=h, work=_region(q))
    for i in range(len(probs)):
        assert torch.equal(Wa[i], Wb[i]) and torch.equal(Za[i], Zb[i]), i


def test_pool_and_region_solves_alternate_on_one_handle(mr3):
    """A handle alternating between its pool and work regions that the caller
    frees in between (each region solve takes its buffers from its own region,
    whatever an earlier solve left in the handle): every solve gives the pool
    solve's bits, the ascending order included."""
    d, e = W.uniform(700, 5, np.float32)
    n = d.size
    h = mr3.Handle(0)
    q = mr3.mr3_workspace_bytes(h, n, mr3.RANGE_ALL, 0, 32)
    W0, Z0 = mr3.solve(_dev(d), _dev(e), handle=h)
    for k in range(3):
        reg = _region(q)
        W1, Z1 = mr3.solve(_dev(d), _dev(e), handle=h, work=reg)
        torch.cuda.synchronize()
        del reg
        torch.cuda.empty_cache()
        assert torch.equal(W0, W1) and torch.equal(Z0, Z1), k
        assert bool(torch.all(W1[1:] >= W1[:-1]))
        W2, Z2 = mr3.solve(_dev(d), _dev(e), handle=h)
        assert torch.equal(W0, W2) and torch.equal(Z0, Z2), k

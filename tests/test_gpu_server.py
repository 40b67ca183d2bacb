"""The serving front end on the device (needs an MI355X): a stream of mixed
requests (both precisions, ALL and INDEX ranges, n from 64 to about 8000,
uniform and noisy 1-2-1 matrices) submitted to one server.  Every result meets
the oracle gates, and matches the same request solved alone: eigenvalues to
the gate, eigenvectors one by one where their gaps pin them and by subspace
angles within groups of close eigenvalues."""
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


def _gates(mr3, h, r, Wt, Zt):
    """Oracle gates for one request's results; returns (R, O).  Up to 600
    eigenpairs every eigenvalue is compared and R, O are evaluated in numpy;
    beyond that 40 sampled eigenvalues are compared and R, O come from the
    device check (FP64 MFMA Gram matrix, FP32 results promoted exactly)."""
    kind, il, iu = r["range"]
    d, e = r["d"], r["e"]
    n = d.size
    eps = M.eps_of(d.dtype)
    d64, e64 = d.astype(np.float64), e.astype(np.float64)
    tn = M.tnorm(d64, e64)
    w = Wt.double().cpu().numpy()
    m = iu - il + 1
    assert w.size == m and np.all(np.diff(w) >= 0)
    if m <= 600:
        hi, lo = oracle.eigvals(d64, e64, il, iu)
        assert np.max(np.abs(w - (hi + lo))) <= 4 * n * eps * tn
        Z = Zt.double().cpu().numpy()
        R, O = M.residual(d64, e64, w, Z), M.orthogonality(Z)
    else:
        for i in np.unique(np.linspace(0, m - 1, 40).astype(int)):
            hi, lo = oracle.eigvals(d64, e64, il + i, il + i)
            assert abs(w[i] - (hi[0] + lo[0])) <= 4 * n * eps * tn, i
        (off, diag), R = mr3.check(_dev(d64), _dev(e64), Wt.double(), Zt.double(), handle=h)
        O = max(off, diag)
    assert R <= 10 * n * eps and O <= 10 * n * eps, (R, O)
    return R, O, tn


def test_server_mixed_stream(mr3):
    reqs = W.served_requests(32, seed=6, lo=64, hi=8192)
    assert max(r["n"] for r in reqs) > 7500
    srv = mr3.Server(mr3.Handle(0), hbm_budget_bytes=4 << 30, max_batch=16)
    tickets = []
    for r in reqs:
        kind, il, iu = r["range"]
        print(f"submit n={r['n']} {np.dtype(r['dtype']).name} {r['kind']} {kind} {il}..{iu}", flush=True)
        tickets.append(srv.submit(_dev(r["d"]), _dev(r["e"]), range=kind, il=il, iu=iu))
    results = [srv.wait(t) for t in tickets]
    srv.close()
    alone = mr3.Handle(0)
    batches = set()
    worst_c, worst_g, ngroups = 0.0, 0.0, 0
    for r, (res, Wt, Zt) in zip(reqs, results):
        batches.add(res["batch_id"])
        kind, il, iu = r["range"]
        d, e = r["d"], r["e"]
        n = d.size
        eps = M.eps_of(d.dtype)
        print(f"check n={n} {np.dtype(r['dtype']).name} {r['kind']} {kind} batch {res['batch_id']}",
              flush=True)
        R, O, tn = _gates(mr3, alone, r, Wt, Zt)
        Wa, Za = mr3.solve(_dev(d), _dev(e), range=kind, il=il, iu=iu, handle=alone)
        Ra, Oa, _ = _gates(mr3, alone, r, Wa, Za)
        c, g, ng = M.alone_vs_mix(Wa.double().cpu().numpy(), Za.double().cpu().numpy(),
                                  Wt.double().cpu().numpy(), Zt.double().cpu().numpy(),
                                  max(R, Ra), max(O, Oa), tn, eps)
        worst_c, worst_g, ngroups = max(worst_c, c / (n * eps)), max(worst_g, g), ngroups + ng
    print(f"batches {len(batches)}; alone vs mix: worst 1-|cos| {worst_c:.3g} n eps, "
          f"groups {ngroups}, worst sin / bound {worst_g:.3g}", flush=True)
    assert len(batches) < len(reqs)  # requests were batched

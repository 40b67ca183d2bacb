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


def test_server_overlaps_a_long_batch(mr3):
    """Continuous batching on the device: while a long FP64 solve runs on one
    slot, short FP32 requests submitted after it are admitted by the other
    slot and complete first; every result meets the oracle gates."""
    srv = mr3.Server(mr3.Handle(0), hbm_budget_bytes=16 << 30, max_batch=8, max_inflight=2)
    dl, el, _ = W.prescribed_spectrum(12000, 3)
    t_long = srv.submit(_dev(dl), _dev(el))
    import time

    time.sleep(0.002)
    shorts = [W.uniform(200 + 10 * i, 40 + i, np.float32) for i in range(4)]
    t_short = [srv.submit(_dev(d), _dev(e)) for d, e in shorts]
    res_short = [srv.wait(t) for t in t_short]
    res_long, Wl, Zl = srv.wait(t_long)
    srv.close()
    first_short = min(r[0]["done_ms"] for r in res_short)
    print(f"long: {res_long['start_ms']:.1f}..{res_long['done_ms']:.1f} slot {res_long['slot']}; "
          f"shorts done at {[round(r[0]['done_ms'], 1) for r in res_short]} slots "
          f"{[r[0]['slot'] for r in res_short]}", flush=True)
    assert first_short < res_long["done_ms"]
    assert any(r[0]["slot"] != res_long["slot"] for r in res_short)
    for (d, e), (res, Wt, Zt) in zip(shorts, res_short):
        n = d.size
        d64, e64 = d.astype(np.float64), e.astype(np.float64)
        hi, lo = oracle.eigvals(d64, e64)
        tn = M.tnorm(d64, e64)
        assert np.max(np.abs(Wt.double().cpu().numpy() - (hi + lo))) <= 4 * n * 2.0 ** -24 * tn
    (off, diag), R = mr3.check(_dev(dl), _dev(el), Wl, Zl)
    n = dl.size
    assert max(off, diag) <= 10 * n * 2.0 ** -53 and R <= 10 * n * 2.0 ** -53

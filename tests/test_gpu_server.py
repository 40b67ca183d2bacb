"""The serving front end on the device (needs an MI355X): a stream of mixed
requests (both precisions, ALL and INDEX ranges, several sizes) submitted to
one server; every result meets the oracle gates and matches a solve of the
same request alone."""
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


def test_server_mixed_stream(mr3):
    reqs = W.served_requests(48, seed=4, lo=64, hi=1024)
    srv = mr3.Server(mr3.Handle(0), hbm_budget_bytes=2 << 30, max_batch=16)
    tickets = []
    for r in reqs:
        kind, il, iu = r["range"]
        print(f"submit n={r['n']} {np.dtype(r['dtype']).name} {kind} {il}..{iu}", flush=True)
        tickets.append(srv.submit(_dev(r["d"]), _dev(r["e"]), range=kind, il=il, iu=iu))
    alone = mr3.Handle(0)
    batches = set()
    for r, t in zip(reqs, tickets):
        res, Wt, Zt = srv.wait(t)
        batches.add(res["batch_id"])
        kind, il, iu = r["range"]
        d, e = r["d"], r["e"]
        n = d.size
        eps = M.eps_of(d.dtype)
        d64, e64 = d.astype(np.float64), e.astype(np.float64)
        tn = M.tnorm(d64, e64)
        w = Wt.double().cpu().numpy()
        assert w.size == iu - il + 1
        hi, lo = oracle.eigvals(d64, e64, il, iu)
        assert np.max(np.abs(w - (hi + lo))) <= 4 * n * eps * tn
        Z = Zt.double().cpu().numpy()
        assert M.residual(d64, e64, w, Z) <= 10 * n * eps
        assert M.orthogonality(Z) <= 10 * n * eps
        wa, _ = mr3.solve(_dev(d), _dev(e), range=kind, il=il, iu=iu, vectors=False, handle=alone)
        assert np.max(np.abs(wa.double().cpu().numpy() - w)) <= 8 * n * eps * tn
    srv.close()
    print("batches", len(batches), flush=True)
    assert len(batches) < len(reqs)  # requests were batched

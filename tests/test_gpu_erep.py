"""The e-representation without cached derived data (mr3_params.derive_lld,
Sec. 3.2 "Choice of representations"): tree nodes keep only d in y and form
lld = e^2 / d from the block's off-diagonals where rows are read.  The
quotient is formed by the formula that stores it otherwise, so every result
is bitwise equal to the stored variant's, on every path that reads lld in y:
the RQI sweeps, the child transforms, the bracket checks and refinement in y
(non-strict children, gaptol below what binary64 resolves, refined cluster
ends) and the bisection fallback of RQI.  The workspace sizes shrink."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr3():
    import paper_1304_1864_amd as lib

    lib.load_library()
    return lib


def _solve_both(mr3, d, e, prec, **kw):
    out = []
    for derive in (0, 1):
        h = mr3.Handle(0)
        h.set_params(precision=prec, derive_lld=derive, **kw)
        Wg, Zg = mr3.solve(torch.from_numpy(d).to("cuda:0"), torch.from_numpy(e).to("cuda:0"), handle=h)
        torch.cuda.synchronize()
        out.append((Wg.cpu().numpy(), Zg.contiguous().cpu().numpy(), h.stats()))
        h.close()
    return out


CASES = [
    ("prescribed n=5000 fp64 (child clusters, non-strict children)", 64, {}),
    ("glued Wilkinson n=4096 fp64", 64, {}),
    ("1-2-1 + noise n=8192 fp32 (a cluster of 136)", 32, {}),
    ("prescribed n=2000 fp64, gaptol 1e-13 (brackets refined in y)", 64, {"gaptol": 1e-13}),
    ("glued Wilkinson n=336 fp64, cluster ends refined in y", 64, {"refine_ends": 1}),
    ("prescribed n=600 fp64, RQI bisection fallback forced", 64, {"force_rqi_fallback": 1}),
]


def _case(name):
    if name.startswith("prescribed n=5000"):
        return W.prescribed_spectrum(5000, 3)[:2]
    if name.startswith("glued Wilkinson n=4096"):
        return W.glued_wilkinson(4096)
    if name.startswith("1-2-1"):
        return W.toeplitz_121_noisy(8192, 4, 1e-6, np.float32)
    if name.startswith("prescribed n=2000"):
        return W.prescribed_spectrum(2000, 2)[:2]
    if name.startswith("glued Wilkinson n=336"):
        return W.glued_wilkinson(336)
    return W.prescribed_spectrum(600, 1)[:2]


@pytest.mark.parametrize("name,prec,kw", CASES, ids=[c[0].split(" (")[0] for c in CASES])
def test_derived_lld_is_bitwise_equal(mr3, name, prec, kw):
    d, e = _case(name)
    print("e-representation:", name, flush=True)
    (w0, z0, s0), (w1, z1, s1) = _solve_both(mr3, d, e, prec, **kw)
    assert np.array_equal(w0, w1) and np.array_equal(z0, z1)
    for key in ("n_clusters", "d_max", "n_fallbacks", "n_y_refined", "n_rqi_iters"):
        assert s0[key] == s1[key], key
    print("   clusters", s1["n_clusters"], "d_max", s1["d_max"], "y-refined", s1["n_y_refined"],
          "fallbacks", s1["n_fallbacks"], flush=True)


def test_derived_lld_batched_and_workspace(mr3):
    probs = W.batch_normal(300, 32, 1024, seed=5, dtype=np.float64)
    res = []
    for derive in (0, 1):
        h = mr3.Handle(0)
        h.set_params(precision=64, derive_lld=derive)
        Ws, Zs = mr3.solve_batched([torch.from_numpy(p[0]).to("cuda:0") for p in probs],
                                   [torch.from_numpy(p[1]).to("cuda:0") for p in probs], handle=h)
        torch.cuda.synchronize()
        res.append([(w.cpu().numpy(), z.contiguous().cpu().numpy()) for w, z in zip(Ws, Zs)])
        full = mr3.mr3_workspace_bytes(h, 20000, mr3.RANGE_ALL, 0, 64)
        low = mr3.mr3_workspace_min_bytes(h, 20000, mr3.RANGE_ALL, 0, 64)
        res[-1].append((full, low))
        h.close()
    for (wa, za), (wb, zb) in zip(res[0][:-1], res[1][:-1]):
        assert np.array_equal(wa, wb) and np.array_equal(za, zb)
    (f0, l0), (f1, l1) = res[0][-1], res[1][-1]
    print("workspace n=20000 fp64: full", f0, "->", f1, "minimum", l0, "->", l1, flush=True)
    assert f1 < f0 and l1 < l0

"""Batched solves on the device (needs an MI355X): one ``mr3_solve_batched``
call over many independent problems of mixed sizes and ranges must meet the
same gates as single solves, and agree with them."""
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


def _ranges_for(sizes, seed):
    """ALL for most problems, an INDEX window for some, a VALUE window for a few."""
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        u = rng.uniform()
        if u < 0.6 or n < 4:
            out.append(("all", 0.0, 0.0, 1, n))
        elif u < 0.85:
            m = max(1, int(np.ceil(0.1 * n)))
            il = int(rng.integers(1, n - m + 2))
            out.append(("index", 0.0, 0.0, il, il + m - 1))
        else:
            vl = float(rng.uniform(-1.5, 0.0))
            out.append(("value", vl, vl + float(rng.uniform(0.2, 1.5)), 1, n))
    return out


def _check_problem(d, e, rng, w, Z, tag):
    n = d.size
    eps = M.eps_of(d.dtype)
    d64, e64 = d.astype(np.float64), e.astype(np.float64)
    kind, vl, vu, il, iu = rng
    if kind == "value":
        il, iu = oracle.count(d64, e64, vl) + 1, oracle.count(d64, e64, vu)
    assert w.size == max(iu - il + 1, 0), (tag, w.size, il, iu)
    if w.size == 0:
        return
    tn = M.tnorm(d64, e64)
    hi, lo = oracle.eigvals(d64, e64, il, iu)
    err = float(np.max(np.abs(w - (hi + lo))))
    assert err <= 4 * n * eps * tn, (tag, err)
    if Z is not None:
        R = M.residual(d64, e64, w, Z)
        O = M.orthogonality(Z)
        assert R <= 10 * n * eps, (tag, "residual", R)
        assert O <= 10 * n * eps, (tag, "orthogonality", O)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batched_mixed_sizes_and_ranges(mr3, dtype):
    probs = W.batch_normal(40, 32, 512, seed=3, dtype=dtype)
    # edge problems inside the batch: sizes 1 and 2, a split matrix, 1-2-1
    d1, e1 = W.uniform(1, 7, dtype)
    d2, e2 = W.uniform(2, 8, dtype)
    ds, es = W.uniform(60, 9, dtype)
    es[19] = 0.0
    probs += [(d1, e1[:0]), (d2, e2[:1]), (ds, es), W.toeplitz_121(200, dtype)]
    sizes = [p[0].size for p in probs]
    ranges = _ranges_for(sizes, 11)
    kinds = {"all": 0, "value": 1, "index": 2}
    desc = [(kinds[r[0]], r[1], r[2], r[3], r[4]) for r in ranges]
    print(f"batched {len(probs)} problems dtype={np.dtype(dtype).name} sum n={sum(sizes)}", flush=True)
    h = mr3.Handle(0)
    Wb, Zb = mr3.solve_batched([_dev(p[0]) for p in probs], [_dev(p[1]) for p in probs],
                               ranges=desc, handle=h)
    torch.cuda.synchronize()
    for i, (p, r) in enumerate(zip(probs, ranges)):
        w = Wb[i].double().cpu().numpy()
        Z = Zb[i].double().cpu().numpy()
        _check_problem(p[0], p[1], r, w, Z, f"problem {i} n={p[0].size} range={r}")
        # the same problem solved alone agrees to the eigenvalue gate
        ws, _ = mr3.solve(_dev(p[0]), _dev(p[1]), range=r[0], vl=r[1], vu=r[2], il=r[3], iu=r[4],
                          vectors=False, handle=h)
        ws = ws.double().cpu().numpy()
        assert ws.size == w.size
        if w.size:
            n = p[0].size
            tn = M.tnorm(p[0].astype(np.float64), p[1].astype(np.float64))
            assert np.max(np.abs(ws - w)) <= 8 * n * M.eps_of(dtype) * tn, i


def test_batched_values_only_and_empty(mr3):
    probs = W.batch_normal(16, 32, 256, seed=5, dtype=np.float32)
    Wb, Zb = mr3.solve_batched([_dev(p[0]) for p in probs], [_dev(p[1]) for p in probs],
                               vectors=False)
    assert Zb is None
    for i, p in enumerate(probs):
        _check_problem(p[0], p[1], ("all", 0.0, 0.0, 1, p[0].size), Wb[i].double().cpu().numpy(),
                       None, f"values-only problem {i}")
    # a value window holding no eigenvalue gives m = 0 for that problem
    d, e = W.uniform(100, 2, np.float64)
    Wb, Zb = mr3.solve_batched([_dev(d), _dev(d)], [_dev(e), _dev(e)],
                               ranges=[(1, 10.0, 11.0, 1, 100), (0, 0.0, 0.0, 1, 100)])
    assert Wb[0].numel() == 0 and Wb[1].numel() == 100


def _device_gates(mr3, d, e, Wt, Zt, h):
    """(O, R) of one problem's results on the device: the FP64 MFMA Gram
    matrix and the residual kernel, with FP32 results promoted exactly."""
    (off, diag), res = mr3.check(_dev(d.astype(np.float64)), _dev(e.astype(np.float64)),
                                 Wt.double(), Zt.double(), handle=h)
    return max(off, diag), res


def test_batched_c3_shape(mr3):
    """The full 4096-problem batch (n log-uniform in [32, 1024], N(0,1),
    FP32): all problems solved in one call; residual and orthogonality of
    every problem on the device, eigenvalues of 64 problems against the
    oracle."""
    probs = W.batch_normal(4096, 32, 1024, seed=0, dtype=np.float32)
    sizes = np.array([p[0].size for p in probs])
    assert int(sizes.sum()) == 1157710
    print("batched C3 shape: 4096 problems, sum n", int(sizes.sum()), flush=True)
    h = mr3.Handle(0)
    Wb, Zb = mr3.solve_batched([_dev(p[0]) for p in probs], [_dev(p[1]) for p in probs], handle=h)
    torch.cuda.synchronize()
    st = h.stats()
    print("   sliced roots", st["n_sliced_roots"], "singleton-first levels", st["n_singleton_first_levels"],
          flush=True)
    assert st["n_sliced_roots"] > 0 and st["n_singleton_first_levels"] > 0
    eps = 2.0 ** -24
    worst_o = worst_r = 0.0
    for i in range(4096):
        n = int(sizes[i])
        assert Wb[i].numel() == n
        assert bool((Wb[i][1:] >= Wb[i][:-1]).all())
        O, R = _device_gates(mr3, probs[i][0], probs[i][1], Wb[i], Zb[i], h)
        assert O <= 10 * n * eps and R <= 10 * n * eps, (i, O, R)
        worst_o, worst_r = max(worst_o, O / (n * eps)), max(worst_r, R / (n * eps))
    print(f"   worst O {worst_o:.3g} n eps, worst R {worst_r:.3g} n eps", flush=True)
    for i in np.linspace(0, 4095, 64).astype(int):
        p = probs[i]
        _check_problem(p[0], p[1], ("all", 0.0, 0.0, 1, p[0].size), Wb[i].double().cpu().numpy(),
                       None, f"C3 problem {i}")


def test_batched_fp64_small_roots_throughput_regime(mr3):
    """An FP64 (double-double) batch large enough to take the paths of the
    throughput-bound regime: 1600 roots of 32 to 256 rows hold more than
    28,800 wanted eigenvalues, so the root multisection runs at two lanes per
    eigenvalue or fewer and roots with at least 16 wanted eigenvalues are
    sliced one workgroup each; and more than 4096 node-pure RQI chunks, so
    each level's singleton work is forked before its cluster work (32 glued
    Wilkinson problems of 84 rows make sure the first level has clusters).
    Residual and orthogonality of every problem on the device, eigenvalues and
    vectors of 24 problems against the oracle."""
    probs = W.batch_normal(1600, 32, 256, seed=21, dtype=np.float64)
    probs[::50] = [W.glued_wilkinson(84) for _ in probs[::50]]
    sizes = np.array([p[0].size for p in probs])
    print("fp64 small-root batch: sum n", int(sizes.sum()), flush=True)
    h = mr3.Handle(0)
    Wb, Zb = mr3.solve_batched([_dev(p[0]) for p in probs], [_dev(p[1]) for p in probs], handle=h)
    torch.cuda.synchronize()
    st = h.stats()
    print("   sliced roots", st["n_sliced_roots"], "singleton-first levels", st["n_singleton_first_levels"],
          "clusters", st["n_clusters"], flush=True)
    assert st["n_sliced_roots"] > 0 and st["n_singleton_first_levels"] > 0
    eps = 2.0 ** -53
    for i, (d, e) in enumerate(probs):
        n = d.size
        O, R = _device_gates(mr3, d, e, Wb[i], Zb[i], h)
        assert O <= 10 * n * eps and R <= 10 * n * eps, (i, O, R)
    for i in np.linspace(0, len(probs) - 1, 24).astype(int):
        d, e = probs[i]
        _check_problem(d, e, ("all", 0.0, 0.0, 1, d.size), Wb[i].cpu().numpy(), Zb[i].cpu().numpy(),
                       f"fp64 small-root problem {i}")
        hi, lo = oracle.eigvals(d, e)
        Zr = oracle.eigvecs(d, e, hi, lo)
        tn = M.tnorm(d, e)
        R = M.residual(d, e, Wb[i].cpu().numpy(), Zb[i].cpu().numpy())
        ratio, worst = M.subspace_sines(hi + lo, Zr, Zb[i].cpu().numpy(), R, tn, 1e-8 * tn)
        assert ratio <= 1.0, (i, worst, ratio)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_deterministic(mr3, dtype):
    """The same call twice gives bitwise-equal eigenvalues and eigenvectors
    (single solves with clusters, and a batch): the perturbation comes from a
    counter-based generator keyed by the row, and no kernel accumulates in an
    order that depends on scheduling."""
    h = mr3.Handle(0)
    if dtype == np.float64:
        d, e = W.glued_wilkinson(336)
    else:
        d, e = W.toeplitz_121_noisy(2000, 3, 1e-6, np.float32)
    W0, Z0 = mr3.solve(_dev(d), _dev(e), handle=h)
    W1, Z1 = mr3.solve(_dev(d), _dev(e), handle=h)
    assert torch.equal(W0, W1) and torch.equal(Z0, Z1)
    probs = W.batch_normal(64, 32, 400, seed=8, dtype=dtype)
    ds, es = [_dev(p[0]) for p in probs], [_dev(p[1]) for p in probs]
    Wa, Za = mr3.solve_batched(ds, es, handle=h)
    Wc, Zc = mr3.solve_batched(ds, es, handle=mr3.Handle(0))
    for i in range(len(probs)):
        assert torch.equal(Wa[i], Wc[i]) and torch.equal(Za[i], Zc[i]), i


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batched_dqds_initial_values(mr3, dtype):
    """dqds initial values in a batch: every problem whose whole spectrum is
    wanted starts from dqds (one lane per root), the others from bisection;
    all meet the gates."""
    probs = W.batch_normal(48, 32, 700, seed=13, dtype=dtype)
    ranges = _ranges_for([p[0].size for p in probs], 17)
    kinds = {"all": 0, "value": 1, "index": 2}
    desc = [(kinds[r[0]], r[1], r[2], r[3], r[4]) for r in ranges]
    h = mr3.Handle(0)
    h.set_params(precision=32 if dtype == np.float32 else 64, initial=mr3.MR3_INITIAL_DQDS)
    print(f"batched dqds {len(probs)} problems dtype={np.dtype(dtype).name}", flush=True)
    Wb, Zb = mr3.solve_batched([_dev(p[0]) for p in probs], [_dev(p[1]) for p in probs],
                               ranges=desc, handle=h)
    torch.cuda.synchronize()
    whole = sum(1 for r in ranges if r[0] == "all")
    assert h.stats()["n_dqds_roots"] >= whole
    for i, (p, r) in enumerate(zip(probs, ranges)):
        _check_problem(p[0], p[1], r, Wb[i].double().cpu().numpy(), Zb[i].double().cpu().numpy(),
                       f"dqds problem {i} n={p[0].size} range={r}")


def test_batched_large_and_small_roots(mr3):
    """A batch mixing a root large enough to be sliced (n = 2500) with small
    roots and a split problem, all pairs and an index window: the same gates
    against the oracle, and the same eigenvalues as solving each alone."""
    dl, el, _ = W.prescribed_spectrum(2500, 3)
    ds, es = W.uniform(90, 4, np.float64)
    es[29] = 0.0
    es[59] = 1e-300
    probs = [(dl, el), W.uniform(300, 5, np.float64), W.toeplitz_121(200, np.float64), (ds, es)]
    for ranges in ([("all", 0.0, 0.0, 1, p[0].size) for p in probs],
                   [("index", 0.0, 0.0, 700, 1300), ("all", 0.0, 0.0, 1, 300),
                    ("index", 0.0, 0.0, 1, 20), ("all", 0.0, 0.0, 1, 90)]):
        kinds = {"all": 0, "value": 1, "index": 2}
        desc = [(kinds[r[0]], r[1], r[2], r[3], r[4]) for r in ranges]
        print(f"batched large+small ranges={[r[0] for r in ranges]}", flush=True)
        h = mr3.Handle(0)
        Wb, Zb = mr3.solve_batched([_dev(p[0]) for p in probs], [_dev(p[1]) for p in probs],
                                   ranges=desc, handle=h)
        torch.cuda.synchronize()
        for i, (p, r) in enumerate(zip(probs, ranges)):
            w = Wb[i].double().cpu().numpy()
            _check_problem(p[0], p[1], r, w, Zb[i].double().cpu().numpy(),
                           f"problem {i} n={p[0].size} range={r}")
            ws, _ = mr3.solve(_dev(p[0]), _dev(p[1]), range=r[0], il=r[3], iu=r[4], vectors=False,
                              handle=h)
            tn = M.tnorm(p[0], p[1])
            assert np.max(np.abs(ws.double().cpu().numpy() - w)) <= 8 * p[0].size * 2.0 ** -53 * tn, i


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_resident_boundary(mr3, dtype):
    """Roots of 1024 rows stay resident in LDS for the whole multisection (and
    a batch of such roots uses one-wave workgroups), roots of 1025 rows stream
    through the staged windows: single solves on both sides of the boundary,
    and a batch mixing them with a small root (four-wave workgroups, resident
    and staged nodes side by side), all against the oracle."""
    probs = [W.uniform(1024, 11, dtype), W.uniform(1025, 12, dtype), W.uniform(33, 13, dtype)]
    for d, e in probs[:2]:
        n = d.size
        print(f"resident boundary single n={n} dtype={np.dtype(dtype).name}", flush=True)
        Wg, Zg = mr3.solve(_dev(d), _dev(e))
        torch.cuda.synchronize()
        _check_problem(d, e, ("all", 0.0, 0.0, 1, n), Wg.double().cpu().numpy(),
                       Zg.double().cpu().numpy(), f"single n={n}")
    for group in (probs[:1] + probs[2:], probs):
        sizes = [p[0].size for p in group]
        print(f"resident boundary batch sizes={sizes} dtype={np.dtype(dtype).name}", flush=True)
        Wb, Zb = mr3.solve_batched([_dev(p[0]) for p in group], [_dev(p[1]) for p in group])
        torch.cuda.synchronize()
        for i, (d, e) in enumerate(group):
            _check_problem(d, e, ("all", 0.0, 0.0, 1, d.size), Wb[i].double().cpu().numpy(),
                           Zb[i].double().cpu().numpy(), f"batch {sizes} problem {i}")

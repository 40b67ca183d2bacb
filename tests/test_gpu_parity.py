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
    out = {"eig_err": err / (n * eps * tn) if tn > 0 else err}
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


def test_check_kernel_matches_numpy(mr3):
    """The FP64 MFMA Gram-matrix check agrees with numpy on a small case."""
    for n, dt in ((700, np.float64), (2500, np.float32)):
        d, e = W.uniform(n, 12, dt)
        Wg, Zg = mr3.solve(_dev(d), _dev(e))
        d, e = d.astype(np.float64), e.astype(np.float64)
        Wg, Zg = Wg.double(), Zg.double()
        (off, diag), res = mr3.check(_dev(d), _dev(e), Wg, Zg)
        Z = Zg.cpu().numpy()
        G = Z.T @ Z
        off_np = np.max(np.abs(G - np.diag(np.diag(G))))
        diag_np = np.max(np.abs(np.diag(G) - 1))
        res_np = M.residual(d, e, Wg.cpu().numpy(), Z)
        assert abs(off - off_np) <= 2 * n * 2.0 ** -53
        assert abs(diag - diag_np) <= 2 * n * 2.0 ** -53
        # both residuals are FP64 evaluations of T z - lambda z: each component
        # carries a rounding error of about 3 eps ||T||_1 |z_k|, so the two
        # 1-norms (relative to ||T||_1) may differ by up to 6 eps ||z||_1 <=
        # 6 eps sqrt(n)
        assert abs(res - res_np) <= 6 * 2.0 ** -53 * np.sqrt(n)


def test_prescribed_child_clusters_regression(mr3):
    """n=5000 prescribed spectrum: many clusters whose children needed a
    twist move; both lanes of a pair must agree on the twist index."""
    d, e, _ = W.prescribed_spectrum(5000, 0)
    h = mr3.Handle(0)
    run_case(mr3, d, e, handle=h)
    st = h.stats()
    assert st["n_clusters"] > 0 and st["d_max"] >= 1


@pytest.mark.slow
def test_glued_wilkinson_4096(mr3):
    d, e = W.glued_wilkinson(4096)
    n = d.size
    h = mr3.Handle(0)
    Wg, Zg = mr3.solve(_dev(d), _dev(e), handle=h)
    w = Wg.cpu().numpy()
    hi, lo = oracle.eigvals(d, e)
    tn = M.tnorm(d, e)
    eps = 2.0 ** -53
    assert np.max(np.abs(w - (hi + lo))) <= 4 * n * eps * tn
    (off, diag), res = mr3.check(_dev(d), _dev(e), Wg, Zg, handle=h)
    assert max(off, diag) <= 10 * n * eps and res <= 10 * n * eps
    st = h.stats()
    print("wilkinson 4096", st["n_clusters"], st["largest_cluster"], st["d_max"], off, diag, res, flush=True)
    # per-group subspace angles against oracle inverse iteration (groups of up
    # to 390 copies of one W21+ eigenvalue, orthogonalised in the oracle)
    Zr = oracle.eigvecs(d, e, hi, lo)
    ratio, worst = M.subspace_sines(hi + lo, Zr, Zg.cpu().numpy(), res, tn, 1e-8 * tn,
                                    O=max(off, diag))
    print("wilkinson 4096 subspace angles: worst sin", worst, "ratio", ratio, flush=True)
    assert ratio <= 1.0


def _sampled_vectors_vs_oracle(d, e, Zg, w, il, idx):
    """Eigenvectors at positions idx (0-based in the computed range starting at
    index il) against oracle inverse iteration, each within the Gap Theorem
    bound of its own residual and the oracle gaps to its neighbours.  Returns
    (worst sin, worst sin / bound)."""
    n = d.size
    Z = Zg[:, torch.as_tensor(np.asarray(idx), device=Zg.device)].double().cpu().numpy()
    worst, worst_ratio = 0.0, 0.0
    for k, i in enumerate(idx):
        j = il + int(i)  # 1-based index of the eigenvalue
        lo_j, hi_j = max(1, j - 1), min(n, j + 1)
        h3, l3 = oracle.eigvals(d, e, lo_j, hi_j)
        c = j - lo_j
        zr = oracle.eigvecs(d, e, h3[c:c + 1], l3[c:c + 1])[:, 0]
        others = [h3[q] + l3[q] for q in range(h3.size) if q != c]
        s, bound = M.gap_theorem_sine(d, e, w[i], Z[:, k], zr, others)
        bound += 2.0 ** -52  # rounding of the oracle vector to binary64
        worst = max(worst, s)
        worst_ratio = max(worst_ratio, s / bound)
        assert s <= bound, (j, s, bound)
    return worst, worst_ratio


@pytest.mark.slow
def test_prescribed_20000_sampled(mr3):
    """Full size of the benchmark workload: all eigenpairs and the subset
    il=1..2000; eigenvalues at sampled indices against the oracle, residual
    and orthogonality of everything on the device, and sampled eigenvectors
    against oracle inverse iteration within the Gap Theorem bound: at both
    ends of the spectrum, across it, and inside the run of tiny eigenvalues
    |lambda| < 1e-7 around zero, whose vectors come from shifted child
    representations (depth 1)."""
    n = 20000
    d, e, lam = W.prescribed_spectrum(n, 0)
    tn = M.tnorm(d, e)
    eps = 2.0 ** -53
    h = mr3.Handle(0)
    dg, eg = _dev(d), _dev(e)
    srt = np.sort(lam)
    tiny = np.nonzero(np.abs(srt) < 1e-7)[0]
    assert tiny.size > 1000
    for rng, il, iu in (("all", 1, n), ("index", 1, 2000)):
        Wg, Zg = mr3.solve(dg, eg, range=rng, il=il, iu=iu, handle=h)
        w = Wg.cpu().numpy()
        m = iu - il + 1
        assert w.size == m and np.all(np.diff(w) >= 0)
        st = h.stats()
        idx = np.unique(np.linspace(0, m - 1, 48).astype(int))
        for i in idx:
            hi, lo = oracle.eigvals(d, e, il + i, il + i)
            assert abs(w[i] - (hi[0] + lo[0])) <= 4 * n * eps * tn, (rng, i)
        (off, diag), res = mr3.check(dg, eg, Wg, Zg, handle=h)
        print(rng, "O", off, diag, "R", res, "gate", 10 * n * eps, st["n_fallbacks"], flush=True)
        assert max(off, diag) <= 10 * n * eps and res <= 10 * n * eps
        vidx = [0, 1, 2, 3, m - 4, m - 3, m - 2, m - 1]
        vidx += list(np.linspace(4, m - 5, 8).astype(int))
        if rng == "all":
            assert st["d_max"] >= 1
            vidx += list(tiny[np.linspace(0, tiny.size - 1, 16).astype(int)])
        worst, ratio = _sampled_vectors_vs_oracle(d, e, Zg, w, il, sorted(set(int(v) for v in vidx)))
        print(rng, "sampled vectors: worst sin", worst, "worst sin / bound", ratio, flush=True)


@pytest.mark.slow
@pytest.mark.parametrize("case", ["uniform-2048", "uniform-4096", "121noisy-8192"])
def test_fp32_large_single(mr3, case):
    """FP32 single solves beyond the sizes of the small parity cases: every
    eigenvalue against the oracle, residual and orthogonality of all pairs on
    the device (FP32 results promoted exactly to FP64), every eigenvector
    against oracle inverse iteration through per-group subspace angles.  The
    1-2-1 matrix plus N(0, 1e-12) noise at n = 8192 forms a cluster of more
    than a hundred eigenvalues at gaptol 1e-5, so it runs through shifted
    child representations and long binary64 sweeps with storage rebasing."""
    kind, n = case.split("-")
    n = int(n)
    if kind == "uniform":
        d, e = W.uniform(n, 30 + n // 1024, np.float32)
    else:
        d, e = W.toeplitz_121_noisy(n, 33, 1e-6, np.float32)
    print(f"fp32 single {case}", flush=True)
    h = mr3.Handle(0)
    Wg, Zg = mr3.solve(_dev(d), _dev(e), handle=h)
    torch.cuda.synchronize()
    st = h.stats()
    eps = 2.0 ** -24
    d64, e64 = d.astype(np.float64), e.astype(np.float64)
    tn = M.tnorm(d64, e64)
    w = Wg.double().cpu().numpy()
    assert w.size == n and np.all(np.diff(w) >= 0)
    hi, lo = oracle.eigvals(d64, e64)
    ref = hi + lo
    err = float(np.max(np.abs(w - ref)))
    assert err <= 4 * n * eps * tn, err
    (off, diag), R = mr3.check(_dev(d64), _dev(e64), Wg.double(), Zg.double(), handle=h)
    O = max(off, diag)
    assert O <= 10 * n * eps and R <= 10 * n * eps, (O, R)
    Zr = oracle.eigvecs(d64, e64, hi, lo)
    ratio, worst = M.subspace_sines(ref, Zr, Zg.double().cpu().numpy(), R, tn, 1e-8 * tn, O=O)
    print(f"   eig err {err / (n * eps * tn):.3g} n eps |T|, R {R / (n * eps):.3g} n eps, "
          f"O {O / (n * eps):.3g} n eps, worst sin {worst:.3g} (ratio {ratio:.3g}), "
          f"clusters {st['n_clusters']} largest {st['largest_cluster']} d_max {st['d_max']}", flush=True)
    assert ratio <= 1.0
    if kind == "121noisy":
        assert st["largest_cluster"] >= 100 and st["d_max"] >= 1


def test_fault_injection_paths(mr3):
    """Forced least-growth shift candidates (and with them the check of child
    brackets in y) and the forced RQI fallback (bisection in y, then one
    step) still meet every gate."""
    h = mr3.Handle(0)
    d, e = W.glued_wilkinson(336)
    h.set_params(precision=64, force_best_candidate=1)
    run_case(mr3, d, e, handle=h)
    assert h.stats()["n_best_candidate"] > 0
    d, e, _ = W.prescribed_spectrum(600, 1)
    h.set_params(precision=64, force_rqi_fallback=1)
    run_case(mr3, d, e, handle=h)
    assert h.stats()["n_fallbacks"] == 600
    d, e = W.uniform(300, 3, np.float32)
    h.set_params(precision=32, force_rqi_fallback=1)
    run_case(mr3, d, e, handle=h)
    assert h.stats()["n_fallbacks"] == 300


def test_host_reordering_fallback(mr3):
    """The host-side reordering (taken when eigenvalues come out of ascending
    order) forced by reversing every problem's outputs on the device: the
    results equal those of the normal path bit for bit (the permutation of
    columns is exact), single solves of both precisions, a split problem,
    and a batch."""
    h = mr3.Handle(0)
    ref = mr3.Handle(0)
    d_split, e_split = W.uniform(90, 4, np.float64)
    e_split[29] = 0.0
    for d, e in (W.uniform(300, 3, np.float32), W.uniform(200, 4, np.float64), (d_split, e_split)):
        prec = 32 if d.dtype == np.float32 else 64
        h.set_params(precision=prec, force_resort=1)
        ref.set_params(precision=prec)
        W0, Z0 = mr3.solve(_dev(d), _dev(e), handle=ref)
        W1, Z1 = mr3.solve(_dev(d), _dev(e), handle=h)
        assert h.stats()["n_resorted"] == 1
        assert torch.equal(W0, W1) and torch.equal(Z0, Z1)
        W2, _ = mr3.solve(_dev(d), _dev(e), range="index", il=5, iu=40, vectors=False, handle=h)
        W3, _ = mr3.solve(_dev(d), _dev(e), range="index", il=5, iu=40, vectors=False, handle=ref)
        assert torch.equal(W2, W3)
    probs = W.batch_normal(12, 32, 200, seed=17, dtype=np.float64)
    h.set_params(precision=64, force_resort=1)
    ds, es = [_dev(p[0]) for p in probs], [_dev(p[1]) for p in probs]
    Wa, Za = mr3.solve_batched(ds, es, handle=h)
    assert h.stats()["n_resorted"] == 12
    Wb, Zb = mr3.solve_batched(ds, es, handle=ref)
    for i in range(12):
        assert torch.equal(Wa[i], Wb[i]) and torch.equal(Za[i], Zb[i]), i


def test_metamorphic_relations(mr3):
    """Exact relations of the method: scaling T by a power of two scales the
    eigenvalues exactly and leaves the vectors unchanged (the input is
    normalised by a power of two first); flipping signs of off-diagonals
    leaves the eigenvalues unchanged and only flips signs of vector entries
    (the representation holds e^2, the vector products hold the signs);
    reversing the row order gives the same spectrum to the gate."""
    d, e = W.uniform(400, 21, np.float64)
    W0, Z0 = mr3.solve(_dev(d), _dev(e))
    W1, Z1 = mr3.solve(_dev(d * 2.0 ** -7), _dev(e * 2.0 ** -7))
    assert torch.equal(W1 * 2.0 ** 7, W0) and torch.equal(Z1, Z0)
    flips = np.where(np.random.default_rng(5).uniform(size=e.size) < 0.5, -1.0, 1.0)
    W2, Z2 = mr3.solve(_dev(d), _dev(e * flips))
    assert torch.equal(W2, W0) and torch.equal(Z2.abs(), Z0.abs())
    W3, Z3 = mr3.solve(_dev(d[::-1].copy()), _dev(e[::-1].copy()))
    n, tn = d.size, M.tnorm(d, e)
    assert float((W3 - W0).abs().max()) <= 4 * n * 2.0 ** -53 * tn
    R = M.residual(d[::-1].copy(), e[::-1].copy(), W3.cpu().numpy(), Z3.cpu().numpy())
    assert R <= 10 * n * 2.0 ** -53


def test_gaptol_settings(mr3):
    """Non-default gaptol: a smaller value (more parallelism) still meets the
    gates; a value below what binary64 eigenvalue approximation resolves at
    this size, 20 n eps_x (Sec. 3.2), has its brackets refined in y and meets
    every gate against the oracle, vectors included; a value below the lower
    end of eq. (gaptolinterval) is refused; absolute-gap splitting is
    accepted and keeps the gates; an FP32 gaptol of 1e-6."""
    d, e, _ = W.prescribed_spectrum(2000, 2)
    h = mr3.Handle(0)
    h.set_params(precision=64, gaptol=1e-11, gaptol_abs=1e-11)
    run_case(mr3, d, e, handle=h, check_angles=False)
    assert h.stats()["n_y_refined"] == 0
    h.set_params(precision=64, gaptol=1e-13)
    run_case(mr3, d, e, handle=h)
    st = h.stats()
    assert st["n_y_refined"] >= d.size
    print("gaptol 1e-13: y-refined brackets", st["n_y_refined"], "clusters", st["n_clusters"],
          "d_max", st["d_max"], flush=True)
    run_case(mr3, d, e, rng="index", il=300, iu=420, handle=h)
    h.set_params(precision=64, gaptol=1e-14)
    with pytest.raises(mr3.MR3Error) as ei:
        mr3.solve(_dev(d), _dev(e), handle=h)
    assert ei.value.code == mr3.MR3_ERR_GAPTOL
    h.set_params(precision=32, gaptol=1e-6)
    d32, e32 = W.uniform(700, 8, np.float32)
    run_case(mr3, d32, e32, handle=h)


def test_refine_cluster_ends_in_y(mr3):
    """The option that refines each cluster's extreme eigenvalues in y before
    its shift is chosen (the footnote of Sec. 3.2): every gate against the
    oracle on matrices with clusters, shallow and deep trees."""
    h = mr3.Handle(0)
    for name, (d, e), g in (("glued Wilkinson n=336", W.glued_wilkinson(336), 1e-10),
                            ("glued Wilkinson n=336, gaptol 1e-3", W.glued_wilkinson(336), 1e-3),
                            ("prescribed n=3000", W.prescribed_spectrum(3000, 5)[:2], 1e-10),
                            ("prescribed n=3000, gaptol 1e-5", W.prescribed_spectrum(3000, 5)[:2], 1e-5)):
        h.set_params(precision=64, refine_ends=1, gaptol=g)
        print("refine ends:", name, flush=True)
        run_case(mr3, d, e, handle=h)
        st = h.stats()
        print("   clusters", st["n_clusters"], "d_max", st["d_max"], "best", st["n_best_candidate"],
              flush=True)
    h.set_params(precision=32, refine_ends=1)
    d, e = W.toeplitz_121_noisy(3000, 4, 1e-6, np.float32)
    run_case(mr3, d, e, handle=h)
    assert h.stats()["n_clusters"] > 0


def test_dqds_initial_values(mr3):
    """Initial eigenvalues from dqds (one lane per root whose whole spectrum is
    wanted, Sec. 4.1) instead of bisection: the same gates against the oracle,
    the same eigenvalues as the bisection path to the gate, and the stats show
    which roots took dqds.  Subsets and roots above the size limit keep
    bisection."""
    h = mr3.Handle(0)
    ref = mr3.Handle(0)
    d_split, e_split = W.uniform(90, 4, np.float64)
    e_split[29] = 0.0
    e_split[59] = 1e-300
    cases = [
        ("uniform n=200 fp64", W.uniform(200, 3, np.float64), 1),
        ("1-2-1 n=300 fp64", W.toeplitz_121(300, np.float64), 1),
        ("glued Wilkinson n=336", W.glued_wilkinson(336), 1),
        ("uniform n=512 fp32", W.uniform(512, 0, np.float32), 1),
        ("prescribed n=600", W.prescribed_spectrum(600, 1)[:2], 1),
        ("Clement n=101 fp32", W.clement(101, np.float32), 1),
        ("split into three", (d_split, e_split), 3),
        ("n=2 fp64", W.uniform(2, 5, np.float64), 1),
    ]
    for name, (d, e), roots in cases:
        prec = 32 if d.dtype == np.float32 else 64
        h.set_params(precision=prec, initial=mr3.MR3_INITIAL_DQDS)
        print("dqds case", name, flush=True)
        run_case(mr3, d, e, handle=h)
        st = h.stats()
        assert st["n_dqds_roots"] == roots, (name, st["n_dqds_roots"])
        assert d.size < 3 or st["dqds_transforms"] > 0, name
        ref.set_params(precision=prec)
        wb, _ = mr3.solve(_dev(d), _dev(e), vectors=False, handle=ref)
        wd, _ = mr3.solve(_dev(d), _dev(e), vectors=False, handle=h)
        n = d.size
        tn = M.tnorm(d.astype(np.float64), e.astype(np.float64))
        diff = float((wb.double() - wd.double()).abs().max())
        assert diff <= 4 * n * M.eps_of(d.dtype) * tn, (name, diff)
    # a subset, and a root above the size limit, keep bisection
    d, e, _ = W.prescribed_spectrum(600, 1)
    h.set_params(precision=64, initial=mr3.MR3_INITIAL_DQDS)
    run_case(mr3, d, e, rng="index", il=20, iu=80, handle=h)
    assert h.stats()["n_dqds_roots"] == 0
    d, e = W.uniform(mr3.MR3_DQDS_MAX_N + 1, 6, np.float32)
    h.set_params(precision=32, initial=mr3.MR3_INITIAL_DQDS)
    mr3.solve(_dev(d), _dev(e), vectors=False, handle=h)
    assert h.stats()["n_dqds_roots"] == 0
    with pytest.raises(mr3.MR3Error):
        h.set_params(precision=64, initial=7)

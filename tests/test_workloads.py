"""Input generators (CPU only): the shared seeded generators are checked
against their defining constructions."""
import numpy as np

import workloads as W


def test_prescribed_spectrum_matches_lanczos():
    """The O(n^2) rotation reconstruction equals n-step Lanczos with full
    reorthogonalisation on diag(lambda) from the same start vector."""
    for n in (1, 2, 7, 60):
        lam = W.prescribed_eigenvalues(n, 11)
        d, e, lam2 = W.prescribed_spectrum(n, 11)
        assert np.array_equal(lam, lam2)
        rng = np.random.default_rng(11 + 7919)
        v = rng.standard_normal(n)
        a, b = W.lanczos_full_reorth(lam, v / np.linalg.norm(v))
        assert np.max(np.abs(a - d)) < 1e-13
        if n > 1:
            assert np.max(np.abs(b - e)) < 1e-13


def test_prescribed_spectrum_eigenvalues():
    d, e, lam = W.prescribed_spectrum(300, 3)
    ev = np.linalg.eigvalsh(np.diag(d) + np.diag(e, 1) + np.diag(e, -1))
    assert np.max(np.abs(ev - np.sort(lam))) < 1e-13
    assert np.min(np.abs(lam)) >= 1e-8 * (1 - 1e-12)


def test_121_closed_form():
    d, e = W.toeplitz_121(40, np.float64)
    ev = np.linalg.eigvalsh(np.diag(d) + np.diag(e, 1) + np.diag(e, -1))
    assert np.max(np.abs(ev - W.toeplitz_121_eigs(40))) < 1e-13


def test_glued_wilkinson_layout():
    d, e = W.glued_wilkinson(45)
    assert d[0] == 10 and d[10] == 0 and d[20] == 10 and d[21] == 10
    assert e[20] == 1e-10 and e[41] == 1e-10 and e[19] == 1.0
    assert d.dtype == np.float64


def test_generators_are_seeded_and_rounded():
    d1, e1 = W.uniform(100, 4)
    d2, e2 = W.uniform(100, 4)
    assert d1.dtype == np.float32 and np.array_equal(d1, d2) and np.array_equal(e1, e2)
    rng = np.random.default_rng(4)
    assert np.array_equal(d1, rng.uniform(-1, 1, 100).astype(np.float32))
    sizes = W.log_uniform_sizes(4096, 32, 1024, 0)
    assert sizes.min() >= 32 and sizes.max() <= 1024

"""Property-based parity (hypothesis) of the HIP path with the oracle, through
the C ABI: small tridiagonals drawn with zeros (splits), repeated entries,
graded and mixed-scale values and a power-of-two scale over a wide exponent
range, in FP32 and FP64, for all pairs and index windows, each checked
against the oracle at the gates (eigenvalues, residual, orthogonality,
subspace angles).  Draws are derandomized, so a run is reproducible."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from tests.test_gpu_parity import run_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mr3():
    import paper_1304_1864_amd as lib

    lib.load_library()
    return lib


entry = st.one_of(
    st.floats(-1.0, 1.0, allow_nan=False, allow_infinity=False, width=32),
    st.sampled_from([0.0, 1.0, -1.0, 0.5, 2.0 ** -20]),
    st.integers(-20, 20).map(lambda k: float(2.0 ** k)),
)


@st.composite
def problem(draw):
    n = draw(st.one_of(st.integers(1, 40), st.integers(41, 300)))
    prec = draw(st.sampled_from([32, 64]))
    vals = draw(st.lists(entry, min_size=2 * n - 1, max_size=2 * n - 1))
    d = np.array(vals[:n], dtype=np.float64)
    e = np.array(vals[n:], dtype=np.float64)
    k = draw(st.integers(-60, 60) if prec == 32 else st.integers(-500, 500))
    d, e = np.ldexp(d, k), np.ldexp(e, k)
    dt = np.float32 if prec == 32 else np.float64
    window = draw(st.one_of(st.none(), st.tuples(st.integers(1, n), st.integers(1, n))))
    return d.astype(dt), e.astype(dt), window


@settings(max_examples=120, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(problem())
def test_random_problems_against_the_oracle(mr3, pb):
    d, e, window = pb
    if window is None:
        run_case(mr3, d, e)
    else:
        il, iu = min(window), max(window)
        run_case(mr3, d, e, rng="index", il=il, iu=iu)


@st.composite
def batch(draw):
    prec = draw(st.sampled_from([32, 64]))
    dt = np.float32 if prec == 32 else np.float64
    count = draw(st.integers(1, 12))
    probs = []
    for _ in range(count):
        n = draw(st.integers(1, 120))
        vals = draw(st.lists(entry, min_size=2 * n - 1, max_size=2 * n - 1))
        k = draw(st.integers(-30, 30))
        d = np.ldexp(np.array(vals[:n]), k).astype(dt)
        e = np.ldexp(np.array(vals[n:]), k).astype(dt)
        probs.append((d, e))
    return probs


@settings(max_examples=25, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(batch())
def test_random_batches_against_the_oracle(mr3, probs):
    """A batched call of random problems: every problem's eigenpairs within
    the gates against the oracle (eigenvalues) and on their own (residual,
    orthogonality)."""
    import torch

    import oracle
    from tests import metrics as M

    ds = [torch.from_numpy(p[0]).to("cuda:0") for p in probs]
    es = [torch.from_numpy(p[1] if p[0].size > 1 else np.zeros(1, p[0].dtype)).to("cuda:0")
          for p in probs]
    Ws, Zs = mr3.solve_batched(ds, es)
    torch.cuda.synchronize()
    for (d, e), w, Z in zip(probs, Ws, Zs):
        n = d.size
        eps = M.eps_of(d.dtype)
        d64, e64 = d.astype(np.float64), e.astype(np.float64)
        tn = M.tnorm(d64, e64)
        hi, lo = oracle.eigvals(d64, e64 if n > 1 else np.zeros(0))
        w = w.double().cpu().numpy()
        assert w.size == n and np.all(np.diff(w) >= 0)
        assert np.max(np.abs(w - (hi + lo))) <= 4 * n * eps * tn
        Zn = Z.double().cpu().numpy()
        assert M.residual(d64, e64, w, Zn) <= 10 * n * eps
        assert M.orthogonality(Zn) <= 10 * n * eps

"""CPU pins of the device double-double arithmetic (csrc/dd.hpp).

The header's operations are __host__ __device__ and use only correctly
rounded binary64 add, multiply and fma, so a host-only build computes the
same bits as the device.  Every error bound the header states is checked
here against exact rational arithmetic (fractions.Fraction), on random
operands over a wide exponent range and on operands chosen to cancel; the
error-free transformations (TwoSum, FastTwoSum, TwoProd) must be exact, and
every result must be normalised (hi is the rounded value of hi + lo)."""
import ctypes
import os
import shutil
import subprocess
from fractions import Fraction as F

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1304_1864_amd", "csrc")
U = F(1, 2 ** 53)
D2 = ctypes.c_double * 2
OPS = {"add": 0, "add_acc": 1, "sub": 2, "mul": 3, "mul_d": 4, "div": 5, "mul_add": 6,
       "mul_sub": 7, "two_sum": 8, "two_prod": 9, "fast_two_sum": 10}


@pytest.fixture(scope="module")
def ddlib(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    out = str(tmp_path_factory.mktemp("ddshim") / "libddshim.so")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-host-only", "-O2", "-ffp-contract=off",
                           "-fPIC", "-shared", "-I", CSRC, os.path.join(HERE, "dd_shim.cpp"),
                           "-o", out])
    lib = ctypes.CDLL(out)
    lib.dds_op.restype = None
    return lib


def _op(lib, name, a, b=(0.0, 0.0), c=(0.0, 0.0), d=(0.0, 0.0)):
    out = D2()
    lib.dds_op(OPS[name], D2(*a), D2(*b), D2(*c), D2(*d), out)
    return out[0], out[1]


def _val(x):
    return F(x[0]) + F(x[1])


def _norm(hi, lo):
    s = hi + lo
    return s, lo - (s - hi)


def _rand_dd(rng, lo_e=-40, hi_e=40):
    e = int(rng.integers(lo_e, hi_e))
    hi = float(rng.uniform(1.0, 2.0) * 2.0 ** e * rng.choice([-1.0, 1.0]))
    return _norm(hi, float(rng.uniform(-0.5, 0.5)) * float(np.spacing(hi)))


def _near_neg(rng, a, rel=1e-8):
    """A dd close to -a (cancelling sums)."""
    hi = -a[0] * (1.0 + float(rng.uniform(-rel, rel)))
    return _norm(hi, float(rng.uniform(-0.5, 0.5)) * float(np.spacing(hi)))


def _normalised(x):
    return x[0] + x[1] == x[0]


def _cases(seed, count):
    rng = np.random.default_rng(seed)
    for k in range(count):
        a, b, c, d = (_rand_dd(rng) for _ in range(4))
        if k % 3 == 1:
            b = _near_neg(rng, a)
        yield rng, a, b, c, d


def test_error_free_transformations(ddlib):
    for rng, a, b, _, _ in _cases(1, 3000):
        x, y = a[0], b[0]
        s = _op(ddlib, "two_sum", (x, 0.0), (y, 0.0))
        assert _val(s) == F(x) + F(y) and s[0] == x + y
        p = _op(ddlib, "two_prod", (x, 0.0), (y, 0.0))
        assert _val(p) == F(x) * F(y) and p[0] == x * y
        big, small = (x, y) if abs(x) >= abs(y) else (y, x)
        f = _op(ddlib, "fast_two_sum", (big, 0.0), (small, 0.0))
        assert _val(f) == F(big) + F(small)


def test_sums(ddlib):
    worst = {"add": 0.0, "sub": 0.0, "add_acc": 0.0}
    for rng, a, b, _, _ in _cases(2, 6000):
        A, B = _val(a), _val(b)
        r = _op(ddlib, "add", a, b)
        assert _normalised(r)
        err = abs(_val(r) - (A + B)) / (abs(A) + abs(B))
        worst["add"] = max(worst["add"], float(err / U ** 2))
        assert err <= 3 * U ** 2, (a, b)
        r = _op(ddlib, "sub", a, b)
        err = abs(_val(r) - (A - B)) / (abs(A) + abs(B))
        worst["sub"] = max(worst["sub"], float(err / U ** 2))
        assert err <= 3 * U ** 2, (a, b)
        r = _op(ddlib, "add_acc", a, b)
        assert _normalised(r)
        if A + B != 0:
            err = abs(_val(r) - (A + B)) / abs(A + B)
            worst["add_acc"] = max(worst["add_acc"], float(err / U ** 2))
            assert err <= 3 * U ** 2 * (1 + 8 * U), (a, b)
        else:
            assert _val(r) == 0
    print("sums, worst error in u^2:", worst)


def test_products_and_quotient(ddlib):
    worst = {"mul": 0.0, "mul_d": 0.0, "div": 0.0}
    for rng, a, b, _, _ in _cases(3, 6000):
        A, B = _val(a), _val(b)
        r = _op(ddlib, "mul", a, b)
        assert _normalised(r)
        err = abs(_val(r) - A * B) / abs(A * B)
        worst["mul"] = max(worst["mul"], float(err / U ** 2))
        assert err <= 6 * U ** 2 * (1 + 8 * U), (a, b)
        r = _op(ddlib, "mul_d", a, b)
        err = abs(_val(r) - A * F(b[0])) / abs(A * F(b[0]))
        worst["mul_d"] = max(worst["mul_d"], float(err / U ** 2))
        assert err <= 2 * U ** 2 * (1 + 8 * U), (a, b)
        r = _op(ddlib, "div", a, b)
        assert _normalised(r)
        err = abs(_val(r) - A / B) / abs(A / B)
        worst["div"] = max(worst["div"], float(err / U ** 2))
        assert err <= 8 * U ** 2 * (1 + 8 * U), (a, b)
    print("products, worst error in u^2:", worst)


def test_fused_steps(ddlib):
    """mul_add(a, b, c) = a b + c and mul_sub(g, a, t, c) = g a - t c, the
    steps of the continuant recurrences, with operands that cancel (c close
    to -a b, t c close to g a) as well as random ones."""
    worst = {"mul_add": 0.0, "mul_sub": 0.0}
    for rng, a, b, c, d in _cases(4, 6000):
        A, B = _val(a), _val(b)
        if rng.uniform() < 0.4:
            c = _near_neg(rng, _op(ddlib, "mul", a, b), 1e-9)
        C = _val(c)
        r = _op(ddlib, "mul_add", a, b, c)
        assert _normalised(r)
        err = abs(_val(r) - (A * B + C))
        worst["mul_add"] = max(worst["mul_add"], float(err / (abs(A * B) + abs(C)) / U ** 2))
        assert err <= 13 * U ** 2 * abs(A * B) + 3 * U ** 2 * abs(C), (a, b, c)
        if rng.uniform() < 0.4:
            # t c close to g a: t = g a / c rounded
            q = _op(ddlib, "div", _op(ddlib, "mul", a, b), c)
            d = _norm(q[0] * (1.0 + float(rng.uniform(-1e-9, 1e-9))), q[1])
        D = _val(d)
        r = _op(ddlib, "mul_sub", a, b, d, c)
        assert _normalised(r)
        err = abs(_val(r) - (A * B - D * C))
        worst["mul_sub"] = max(worst["mul_sub"], float(err / (abs(A * B) + abs(D * C)) / U ** 2))
        assert err <= 13 * U ** 2 * (abs(A * B) + abs(D * C)), (a, b, d, c)
    print("fused steps, worst error in u^2 (relative to the operand sizes):", worst)

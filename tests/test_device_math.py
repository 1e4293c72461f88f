"""The FP64 exponential and sine/cosine of the trajectory kernels, checked on
the host: their constants are read from the device source and the device's
order of operations is replayed with correctly rounded FMAs (50-digit
arithmetic rounded to double after every operation), against the exact
functions.  Pins the error bounds stated beside the device code."""
import math
import os
import re

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")
mp.mp.dps = 50

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2608_13686_amd", "csrc",
                   "device_common.h")


def constants(func):
    """The dbits(...) literals of one device function, in source order."""
    text = open(SRC).read()
    m = re.search(r"__device__ __forceinline__ \w+ " + func + r"\(.*?\n}\n", text, re.S)
    assert m, func
    return [float(x) for x in re.findall(r"dbits\(([-+0-9.eE]+)\)", m.group(0))]


def fma(a, b, c):
    return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))


def mul(a, b):
    return float(mp.mpf(a) * mp.mpf(b))


def add(a, b):
    return float(mp.mpf(a) + mp.mpf(b))


def exp_neg(y, k):
    """e^{-y} in the device's order: n = rint(-y/ln2) (round half to even),
    two-part reduction, Horner from the highest coefficient, ldexp."""
    nlog2e, ln2, ln2lo, c11, c10, *rest = k
    n = float(np.rint(mul(y, nlog2e)))
    r = float(-mp.mpf(n) * mp.mpf(ln2) - mp.mpf(y))
    r = fma(-n, ln2lo, r)
    q = add(mul(r, c11), c10)
    for c in rest:
        q = fma(q, r, c)
    q = fma(q, r, 1.0)
    q = fma(q, r, 1.0)
    return math.ldexp(q, int(n))


def sincos(x, k):
    two_pi, pio2, pio2lo, s5, s4, s3, s2, s1, s0, c5, c4, c3, c2, c1, c0 = k
    n = float(np.rint(mul(x, two_pi)))
    r = fma(-n, pio2, x)
    r = fma(-n, pio2lo, r)
    z = mul(r, r)
    ps = add(mul(z, s5), s4)
    for c in (s3, s2, s1, s0):
        ps = fma(ps, z, c)
    pc = add(mul(z, c5), c4)
    for c in (c3, c2, c1, c0):
        pc = fma(pc, z, c)
    s_r = fma(mul(r, z), ps, r)
    c_r = fma(mul(z, z), pc, fma(z, -0.5, 1.0))
    q = int(n)
    s0_, c0_ = (c_r, s_r) if q & 1 else (s_r, c_r)
    if q & 2:
        s0_ = -s0_
    if (q + 1) & 2:
        c0_ = -c0_
    return s0_, c0_


def exp_constants():
    """-1/ln2, ln2, its low part, then the fit from the highest coefficient
    (add_k<c10>(mul_k<c11>(r)) names c10 first in the source)."""
    k = constants("exp_neg")
    return k[:3] + [k[4], k[3]] + k[5:]


def sincos_constants():
    """2/pi, the two parts of pi/2, then S and C from the highest coefficient."""
    k = constants("sincos_k")
    return k[:3] + [k[4], k[3]] + k[5:9] + [k[10], k[9]] + k[11:]


def test_constants_found():
    assert len(constants("exp_neg")) == 13
    assert len(constants("sincos_k")) == 15
    # the two-argument form uses the same constants
    assert constants("exp_neg2") == exp_constants()


def test_exp_neg_error_below_stated_bound():
    k = exp_constants()
    rng = np.random.default_rng(5)
    ys = np.concatenate([rng.uniform(0, 60, 1500), rng.uniform(60, 708, 500),
                         np.arange(0, 61) * math.log(2) / 2,  # reduction boundaries
                         [0.0, 1e-300, 1e-12, 700.0, 708.0]])
    worst = 0.0
    for y in ys:
        e, t = exp_neg(float(y), k), mp.exp(-mp.mpf(float(y)))
        worst = max(worst, float(abs(mp.mpf(e) - t) / (t * mp.mpf(2) ** -52)))
    assert worst < 0.7, worst


def test_sincos_error_below_stated_bound():
    k = sincos_constants()
    rng = np.random.default_rng(6)
    xs = np.concatenate([rng.uniform(-4, 4, 800), rng.uniform(-2e4, 2e4, 800),
                         np.arange(-8, 9) * math.pi / 4,  # quadrant edges
                         [0.0, 1e-20, -1e-20, 1e6 + 0.3, -3e8]])
    worst = 0.0
    for x in xs:
        s, c = sincos(float(x), k)
        xm = mp.mpf(float(x))
        worst = max(worst, float(abs(s - mp.sin(xm))), float(abs(c - mp.cos(xm))))
    assert worst < 2.0 ** -52, worst


def test_constants_are_the_committed_generator_output():
    """Every polynomial and reduction constant of the device exponential and
    sine/cosine is what csrc/fit_device_math.py computes (Chebyshev fits in
    40-digit arithmetic, rounded to double)."""
    import importlib.util
    path = os.path.join(os.path.dirname(SRC), "fit_device_math.py")
    spec = importlib.util.spec_from_file_location("fit_device_math", path)
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    want = gen.fits()
    assert exp_constants() == want["exp"]
    assert constants("exp_neg2") == want["exp"]
    text = open(SRC).read()
    m = re.search(r"const double v\[13\] = \{(.*?)\};", text, re.S)
    assert [float(x) for x in m.group(1).replace("\n", " ").split(",")] == want["exp"]
    assert sincos_constants() == want["sincos"]

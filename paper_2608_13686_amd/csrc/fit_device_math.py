"""Generator of the polynomial constants of the device exponential and
sine/cosine in device_common.h (exp_neg, exp_neg2, ExpK, sincos_k).

    python paper_2608_13686_amd/csrc/fit_device_math.py

prints every constant in the order the device code uses it.  The fits are
Chebyshev interpolants (mpmath.chebyfit, 40 significant digits) rounded to
double:

* e^r = 1 + r (1 + r q(r)) on |r| <= ln2/2, q of degree 9 fitted to
  (e^r - 1 - r) / r^2;
* sin r = r + r z S(z), cos r = 1 - z/2 + z^2 C(z) on |r| <= pi/4, z = r^2,
  S and C of degree 5 in z fitted to (sin r / r - 1) / z and
  (cos r - 1 + z/2) / z^2 on z in [0, (pi/4)^2];
* the range reductions: -1/ln2 and ln2 split into a double and the double
  nearest the rest; 2/pi and pi/2 split the same way.

tests/test_device_math.py checks that device_common.h holds exactly these
numbers and that the device's order of operations meets its error bounds.
"""
import mpmath as mp


def split(x):
    """x as a double hi and the double nearest x - hi."""
    hi = float(x)
    return hi, float(x - mp.mpf(hi))


def fits(dps=40):
    mp.mp.dps = dps
    half_ln2 = mp.log(2) / 2

    def q(r):
        return (mp.exp(r) - 1 - r) / r ** 2

    def s(z):
        return (mp.sin(mp.sqrt(z)) / mp.sqrt(z) - 1) / z

    def c(z):
        return (mp.cos(mp.sqrt(z)) - 1 + z / 2) / z ** 2

    zmax = (mp.pi / 4) ** 2
    ln2_hi, ln2_lo = split(mp.log(2))
    pio2_hi, pio2_lo = split(mp.pi / 2)
    return {
        # exponential: -1/ln2, ln2 (hi, lo), q highest degree first
        "exp": [float(-1 / mp.log(2)), ln2_hi, ln2_lo] +
               [float(x) for x in mp.chebyfit(q, [-half_ln2, half_ln2], 10)],
        # sine/cosine: 2/pi, pi/2 (hi, lo), S then C, highest degree first
        "sincos": [float(2 / mp.pi), pio2_hi, pio2_lo] +
                  [float(x) for x in mp.chebyfit(s, [0, zmax], 6)] +
                  [float(x) for x in mp.chebyfit(c, [0, zmax], 6)],
    }


if __name__ == "__main__":
    for name, vals in fits().items():
        print(name)
        for v in vals:
            print(f"  {v!r}")

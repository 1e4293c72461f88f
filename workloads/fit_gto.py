"""Writes ``gto_default.json``: the synthetic Gaussian-type-orbital (GTO) tables
used as the initial orbital psi_0 of the workloads.

The paper expands psi_0 in GTOs fitted to the numerical HOMO of its model
potential (Sec. II.A, the paragraph after the sampling rule; 6-311G for H2,
cc-pV5Z for N2).  Those fitted coefficients are not published, so these
tables are synthetic stand-ins, built here and stated as such:

* each radial factor exp(-kappa r), with kappa = sqrt(2 Ip) (the asymptotic
  decay of a bound state with binding energy Ip), is least-squares fitted in
  the 3D L2 norm by a short sum of s-Gaussians;
* H2 1sigma_g : one s contraction (3 primitives) on each centre, same sign;
* N2 3sigma_g : an s contraction (2 primitives) plus a p contraction along the
  molecular axis (2 primitives, same radial fit) on each centre; the p
  coefficients have opposite sign on the two centres so that the orbital is
  gerade (even under inversion), with the positive p lobe pointing away from
  the partner nucleus; the p part enters with relative amplitude ETA_P;
* the whole orbital is normalised to <psi_0|psi_0> = 1 at its internuclear
  distance R.

This is input preparation, not the method: nothing here is used by the
propagation.  Run ``python workloads/fit_gto.py`` to regenerate the table.
"""
import json
import math
import os

import numpy as np
from scipy.optimize import least_squares

HARTREE_EV = 27.211386245988  # CODATA 2018
ETA_P = 0.6                   # relative amplitude of the N2 p part (synthetic)


def fit_slater(zeta, n_prim):
    """Fit exp(-zeta r) ~ sum_i c_i exp(-a_i r^2) in the 3D L2 norm."""
    r = np.linspace(0.0, 40.0 / zeta, 20001)
    wgt = r * r * (r[1] - r[0])
    target = np.exp(-zeta * r)

    def design(loga):
        return np.exp(-np.outer(r * r, np.exp(loga)))

    def resid(loga):
        B = design(loga)
        sw = np.sqrt(wgt)
        c, *_ = np.linalg.lstsq(B * sw[:, None], target * sw, rcond=None)
        return (B @ c - target) * sw

    x0 = np.log(np.geomspace(0.08, 3.0, n_prim) * zeta * zeta)
    sol = least_squares(resid, x0, xtol=1e-14, ftol=1e-14, gtol=1e-14)
    a = np.exp(sol.x)
    B = design(sol.x)
    sw = np.sqrt(wgt)
    c, *_ = np.linalg.lstsq(B * sw[:, None], target * sw, rcond=None)
    order = np.argsort(a)
    return a[order], c[order]


def overlap(p1, p2, R):
    """<g1|g2> for primitives (center, l, a, c) with centres at +-R/2 on the axis."""
    (c1, l1, a, ca), (c2, l2, b, cb) = p1, p2
    z1 = R / 2 if c1 == 0 else -R / 2
    z2 = R / 2 if c2 == 0 else -R / 2
    g = a + b
    P = (a * z1 + b * z2) / g
    sss = (math.pi / g) ** 1.5 * math.exp(-a * b / g * (z1 - z2) ** 2)
    if l1 == 0 and l2 == 0:
        val = sss
    elif l1 == 1 and l2 == 0:
        val = (P - z1) * sss
    elif l1 == 0 and l2 == 1:
        val = (P - z2) * sss
    else:
        val = ((P - z1) * (P - z2) + 0.5 / g) * sss
    return ca * cb * val


def normalise(prims, R):
    s = sum(overlap(p, q, R) for p in prims for q in prims)
    k = 1.0 / math.sqrt(s)
    return [(c, l, a, coef * k) for (c, l, a, coef) in prims]


def build():
    out = {}
    # H2: Ip = 15.40 eV (Table II), R = 1.40
    ip = 15.40 / HARTREE_EV
    a, c = fit_slater(math.sqrt(2 * ip), 3)
    prims = [(ctr, 0, float(ai), float(ci)) for ctr in (0, 1) for ai, ci in zip(a, c)]
    out["H2"] = {"R": 1.40, "Ip_eV": 15.40, "prims": normalise(prims, 1.40)}
    # N2: Ip = 15.58 eV (the N2 workloads' value), R = 2.07
    ip = 15.58 / HARTREE_EV
    a, c = fit_slater(math.sqrt(2 * ip), 2)
    prims = []
    for ctr, sgn in ((0, +1.0), (1, -1.0)):
        prims += [(ctr, 0, float(ai), float(ci)) for ai, ci in zip(a, c)]
        prims += [(ctr, 1, float(ai), float(sgn * ETA_P * ci)) for ai, ci in zip(a, c)]
    out["N2"] = {"R": 2.07, "Ip_eV": 15.58, "prims": normalise(prims, 2.07)}
    return out


if __name__ == "__main__":
    tab = build()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gto_default.json")
    with open(path, "w") as f:
        json.dump({"_about": "synthetic GTO tables written by workloads/fit_gto.py; "
                             "prims are [center(0:+R/2 n, 1:-R/2 n), l(0=s,1=p along n), exponent, coefficient]",
                   **tab}, f, indent=1)
    print(json.dumps(tab, indent=1))

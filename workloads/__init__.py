"""Seeded synthetic workload definitions shared by the HIP path, the oracle,
the tests and the benchmark.

This module holds plain numbers only: laser and target parameters, the
synthetic GTO tables, ensemble sizes and seeds, and the seeded generator of
the request stream.  It holds none of the method's arithmetic (no field, no
potential, no sampling transform, no propagation): each side derives those
from these numbers on its own.

Problem dictionaries have the layout::

    {"name": str,
     "laser":  {"lambda_nm", "intensity_wcm2", "n_cycles", "cep"},
     "target": {"R", "Ip" (hartree), "centers": [2 x {"Zinf","dZ","alpha","eps2"}],
                "gto": [(center, l, a, c), ...]},
     "align":  {"kind": "fixed"|"cos2m", "theta", "phi", "m"},
     "dt", "gamma", "w_cut", "sigma_perp", "n_steps" (0 = round(tau/dt)),
     optional "c_max" (> 0: prefactor cap; absent = prefactor fully included)}

Atomic units throughout, except the laser (nm, W/cm^2, cycles, rad).
"""
import copy
import json
import math
import os

import numpy as np

HARTREE_EV = 27.211386245988  # CODATA 2018, eV per hartree

_HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(_HERE, "gto_default.json")) as _f:
    _GTO = json.load(_f)


def gto_table(molecule):
    """Synthetic GTO table (center, l, exponent, coefficient) for 'H2' or 'N2'."""
    return [tuple(p) for p in _GTO[molecule]["prims"]]


def ev_to_hartree(e_ev):
    return e_ev / HARTREE_EV


def _problem(name, laser, R, ip_ev, center, gto, align, dt):
    return {
        "name": name,
        "laser": dict(laser),
        "target": {"R": R, "Ip": ev_to_hartree(ip_ev),
                   "centers": [dict(center), dict(center)], "gto": list(gto)},
        "align": dict(align),
        "dt": dt, "gamma": 1.0, "w_cut": 1e-8, "sigma_perp": 0.3, "n_steps": 0,
    }


# --- the H2 soft-core problem: -0.5/sqrt(|r -+ R/2|^2 + 0.5), R = 1.4,
#     800 nm, 2e14 W/cm^2, 3-cycle sin^2, CEP 0, Ip 15.40 eV (Table II), dt 0.1
H2_SOFTCORE_CENTER = {"Zinf": 0.5, "dZ": 0.0, "alpha": 0.0, "eps2": 0.5}
H2_LASER = {"lambda_nm": 800.0, "intensity_wcm2": 2e14, "n_cycles": 3.0, "cep": 0.0}

# --- the N2 problem: Eq. (7) with the Table I N2 parameters (Z_inf 0.5,
#     Z_0 7.0, alpha 1.67, R 2.07), softened by eps^2 = 0.5; 1200 nm,
#     1.5e14 W/cm^2, 4-cycle sin^2 (the paper's laser, Sec. III.A), Ip 15.58 eV
N2_CENTER = {"Zinf": 0.5, "dZ": 6.5, "alpha": 1.67, "eps2": 0.5}
N2_LASER = {"lambda_nm": 1200.0, "intensity_wcm2": 1.5e14, "n_cycles": 4.0, "cep": 0.0}


def fixed(theta_deg, phi_deg=0.0):
    return {"kind": "fixed", "theta": math.radians(theta_deg), "phi": math.radians(phi_deg), "m": 0}


def cos2m(m=2):
    return {"kind": "cos2m", "theta": 0.0, "phi": 0.0, "m": m}


def h2_softcore(theta_deg=0.0, laser=None, align=None):
    return _problem("H2-softcore", laser or H2_LASER, 1.4, 15.40, H2_SOFTCORE_CENTER,
                    gto_table("H2"), align or fixed(theta_deg), 0.1)


def n2(theta_deg=0.0, laser=None, align=None):
    return _problem("N2-eq7", laser or N2_LASER, 2.07, 15.58, N2_CENTER,
                    gto_table("N2"), align or fixed(theta_deg), 0.05)


def with_changes(prob, **kw):
    """Copy of a problem with top-level or nested ('laser.intensity_wcm2') keys replaced."""
    p = copy.deepcopy(prob)
    for key, val in kw.items():
        d = p
        parts = key.split(".")
        for part in parts[:-1]:
            d = d[part]
        d[parts[-1]] = val
    return p


def free_problem(prob):
    """The same problem with the ion potential switched off (Z_inf = dZ = 0)."""
    p = copy.deepcopy(prob)
    for c in p["target"]["centers"]:
        c["Zinf"] = 0.0
        c["dZ"] = 0.0
    return p


def laser_off(prob):
    p = copy.deepcopy(prob)
    p["laser"]["intensity_wcm2"] = 0.0
    return p


# ---------------------------------------------------------------- workloads
# Sizes and seeds of the five measured workloads.  Each entry: problems,
# trajectories per problem, per-problem seeds.

def workload_h2_fixed():
    """H2 soft-core, fixed alignment parallel to the field, 4096 trajectories, seed 1001."""
    return {"name": "h2-softcore-fixed0-4096", "problems": [h2_softcore(0.0)],
            "n_traj": [4096], "seeds": [1001], "precision": "fp64"}


def workload_n2_fixed(n_traj=1 << 20, precision="fp64"):
    """N2, fixed alignment at 0 and 90 degrees, 1,048,576 trajectories per angle,
    both angles drawing the same (seed 1002) trajectories."""
    return {"name": f"n2-fixed-0-90-{n_traj}", "problems": [n2(0.0), n2(90.0)],
            "n_traj": [n_traj, n_traj], "seeds": [1002, 1002], "precision": precision}


def workload_batched(n_per_problem=32768):
    """H2 and N2 with a cos^4 axis distribution over a 64-laser grid each:
    intensities linspace(1e14, 3e14, 8) x CEPs k*pi/4; 128 x 32,768 = 2^22
    trajectories; seed 1003 mixed with the problem index."""
    probs, seeds = [], []
    intens = np.linspace(1e14, 3e14, 8)
    for mol in ("H2", "N2"):
        for i, inten in enumerate(intens):
            for k in range(8):
                base_laser = H2_LASER if mol == "H2" else N2_LASER
                las = dict(base_laser, intensity_wcm2=float(inten), cep=k * math.pi / 4)
                p = (h2_softcore if mol == "H2" else n2)(laser=las, align=cos2m(2))
                p["name"] = f"{mol}-I{i}-cep{k}"
                probs.append(p)
                seeds.append(1003 * 1000003 + len(seeds))
    return {"name": f"batched-h2n2-cos4-128x{n_per_problem}", "problems": probs,
            "n_traj": [n_per_problem] * len(probs), "seeds": seeds, "precision": "mixed"}


def workload_averaging(mol="H2", n_angles=10):
    """Isotropic alignment average two ways (Sec. III.B, Eq. 5 and Eq. 6):
    'standard': n_angles fixed alignments at the Gauss-Legendre nodes of
    x = cos(theta) on [0, 1] (the homonuclear symmetry theta -> pi - theta
    folds [-1, 1] onto [0, 1]) with weights summing to 1, each run on its own;
    'joint': one problem whose axis is drawn uniformly on the sphere with the
    trajectory (the cos^0 density)."""
    x, w = np.polynomial.legendre.leggauss(n_angles)
    make = h2_softcore if mol == "H2" else n2
    thetas = [math.degrees(math.acos(0.5 * (xi + 1.0))) for xi in x]
    return {"standard": ([make(th) for th in thetas], [0.5 * wi for wi in w]),
            "joint": make(align=cos2m(0)), "thetas_deg": thetas}


def request_stream(n_requests, rate_hz, seed=1004, n_min=10_000, n_max=4_000_000):
    """Seeded Poisson stream of spectrum requests.

    Each request: H2 or N2 (50/50); intensity U[1,4]e14 W/cm^2; wavelength
    U[800,1800] nm; 2..6 cycles; fixed axis (theta ~ U[0,90] deg) or cos^4
    (50/50); trajectory count lognormal (median 2e5) truncated to
    [n_min, n_max].  Returns a list of (arrival_time_s, problem, n_traj, seed).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        mol = "H2" if rng.random() < 0.5 else "N2"
        las = {"lambda_nm": float(rng.uniform(800.0, 1800.0)),
               "intensity_wcm2": float(rng.uniform(1e14, 4e14)),
               "n_cycles": float(rng.integers(2, 7)), "cep": 0.0}
        if rng.random() < 0.5:
            al = fixed(float(rng.uniform(0.0, 90.0)))
        else:
            al = cos2m(2)
        p = (h2_softcore if mol == "H2" else n2)(laser=las, align=al)
        while True:
            n = int(round(math.exp(rng.normal(math.log(2e5), 0.9986))))
            if n_min <= n <= n_max:
                break
        out.append((t, p, n, int(seed * 1000003 + r)))
    return out

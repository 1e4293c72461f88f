"""Pins of the oracle's classical return analysis (long and short
trajectories, Sec. III.C): free-electron returns against the closed-form
orbit, and the 3.17 U_p cutoff of the simple-man model."""
import math

import numpy as np

import workloads as W


def free_orbit(orc, p, k0, q0, p0):
    """q(t_k) of a free electron in the pulse, from the antiderivative of the
    three-carrier form of A: q_z = q0_z + (p0_z - A(t0))(t - t0) + F(t) - F(t0)."""
    w, E0, tau, N = orc.laser(p)
    phi = p["laser"]["cep"]
    Om = 2 * math.pi / tau
    wj = np.array([w, w + Om, w - Om])
    cj = np.array([0.5, 0.25, 0.25])
    a0 = E0 / w
    F = lambda t: a0 * np.sum(cj / wj * np.cos(np.outer(t, wj) + phi), axis=1)
    t = orc.times(p)
    t0 = t[k0]
    _, A0 = orc.field(p, t0)
    qz = q0[2] + (p0[2] - A0) * (t - t0) + F(t) - F(np.array([t0]))[0]
    qx = q0[0] + p0[0] * (t - t0)
    qy = q0[1] + p0[1] * (t - t0)
    return np.stack([qx, qy, qz], axis=1)


def test_free_electron_returns_match_the_closed_form(orc):
    p = W.free_problem(W.n2(0.0))
    w, E0, tau, N = orc.laser(p)
    Ip = p["target"]["Ip"]
    r_ret = 4.0
    rng = np.random.default_rng(11)
    found = 0
    for _ in range(40):
        k0 = int(rng.integers(N // 4, 3 * N // 4))
        E, _ = orc.field(p, orc.time(p, k0))
        if abs(E) < 0.2 * E0:
            continue
        q0 = np.array([0.0, 0.0, -Ip / E])
        p0 = np.array([rng.normal(0, 0.05), 0.0, 0.0])
        k, e = orc.return_step(p, k0, q0, p0, (0, 0, 1), r_ret)
        q = free_orbit(orc, p, k0, q0, p0)
        r = np.linalg.norm(q[k0:], axis=1)
        out = np.nonzero(r >= r_ret)[0]
        ref = -1
        if out.size:
            back = np.nonzero(r[out[0]:] < r_ret)[0]
            if back.size:
                ref = k0 + out[0] + back[0]
        assert k == ref
        if k >= 0:
            found += 1
            t = orc.times(p)
            _, A = orc.field(p, t[k])
            _, A0 = orc.field(p, t[k0])
            pk = p0 + np.array([0, 0, A - A0])
            assert e == pytest_approx(0.5 * pk @ pk, 1e-7)
    assert found > 5


def pytest_approx(x, rel):
    import pytest
    return pytest.approx(x, rel=rel, abs=1e-12)


def test_simple_man_cutoff_3_17_up(orc):
    """Electrons released at rest at the origin of a quasi-monochromatic
    pulse return with at most ~3.17 U_p of kinetic energy."""
    p = W.free_problem(W.h2_softcore(0.0, laser=dict(W.H2_LASER, n_cycles=16.0)))
    p["dt"] = 0.1
    w, E0, tau, N = orc.laser(p)
    Up = E0 * E0 / (4 * w * w)
    T = 2 * math.pi / w
    t = orc.times(p)
    centre = np.nonzero(np.abs(t) < 0.5 * T)[0][::4]
    best = 0.0
    for k0 in centre:
        k, e = orc.return_step(p, int(k0), (0, 0, 0), (0, 0, 0), (0, 0, 1), 0.3)
        if k >= 0:
            best = max(best, e)
    assert 3.0 < best / Up < 3.25

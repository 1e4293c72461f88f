"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
closed form, an invariant, a brute-force or library computation, or a
number the paper prints (``tests/golden/paper_values.json``).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
HARTREE_EV = workloads.HARTREE_EV

with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
    PAPER = json.load(f)


def J6():
    J = np.zeros((6, 6))
    J[:3, 3:] = np.eye(3)
    J[3:, :3] = -np.eye(3)
    return J


# ------------------------------------------------------------------ inputs
def test_workloads_use_paper_tables():
    """Table I / Table II numbers reach the N2 problem and the GTO-fit inputs."""
    t1 = PAPER["table_I_model_potential"]["N2"]
    p = workloads.n2()
    c = p["target"]["centers"][0]
    assert p["target"]["R"] == t1["R"]
    assert c["Zinf"] == t1["Zinf"] and c["Zinf"] + c["dZ"] == t1["Z0"] and c["alpha"] == t1["alpha"]
    h = workloads.h2_softcore()
    assert h["target"]["R"] == PAPER["table_I_model_potential"]["H2"]["R"]
    assert abs(h["target"]["Ip"] * HARTREE_EV - PAPER["table_II_binding_energies_eV"]["H2_HOMO_1sigma_g"]) < 1e-12
    assert h["gamma"] == PAPER["coherent_state_width"]["gamma"]


# ------------------------------------------------------------------- laser
def test_laser_vector_potential_closed(orc):
    p = workloads.n2()
    w, E0, tau, N = orc.laser(p)
    for t in (-tau / 2, tau / 2):
        E, A = orc.field(p, t)
        assert abs(A) < 1e-15
    E, A = orc.field(p, 0.0)
    assert abs(E - E0) < 1e-15  # CEP 0: the field peaks at the pulse centre
    # E = -dA/dt by central differences at many times
    ts = np.linspace(-0.49 * tau, 0.49 * tau, 97)
    h = 1e-4
    Ep, Ap = orc.field(p, ts + h)
    Em, Am = orc.field(p, ts - h)
    E, _ = orc.field(p, ts)
    assert np.max(np.abs(E + (Ap - Am) / (2 * h))) < 1e-9
    # no DC component: int E dt = -(A(tau/2) - A(-tau/2)) = 0
    val, _ = integrate.quad(lambda t: orc.field(p, t)[0], -tau / 2, tau / 2, limit=400)
    assert abs(val) < 1e-10


def test_keldysh_and_cutoff_match_paper(orc):
    """Keldysh ~0.6 (Sec. III.A) and the H2 cutoff near 80 eV (Sec. III.A, Fig. 1)
    from the simple-man return energies in the oracle's field."""
    p = workloads.n2()
    w, E0, tau, N = orc.laser(p)
    Up = E0 ** 2 / (4 * w * w)
    kel_n2 = math.sqrt(p["target"]["Ip"] / (2 * Up))
    ip_h2 = PAPER["table_II_binding_energies_eV"]["H2_HOMO_1sigma_g"] / HARTREE_EV
    kel_h2 = math.sqrt(ip_h2 / (2 * Up))
    for k in (kel_n2, kel_h2):
        assert abs(k - PAPER["laser_main"]["keldysh_approx"]) < 0.05
    t = np.linspace(-tau / 2, tau / 2, 60001)
    E, A = orc.field(p, t)
    X = integrate.cumulative_trapezoid(A, t, initial=0.0)
    kmax = 0.0
    for i0 in range(0, t.size - 100, 60):
        x = X[i0:] - X[i0] - A[i0] * (t[i0:] - t[i0])
        s = np.sign(x[20:])
        idx = np.nonzero(s[1:] != s[:-1])[0]
        if idx.size:
            j = i0 + 21 + idx[0]
            kmax = max(kmax, 0.5 * (A[j] - A[i0]) ** 2)
    cutoff = (kmax + ip_h2) * HARTREE_EV
    assert abs(cutoff - PAPER["h2_spectrum"]["cutoff_eV_approx"]) < 7.0


def test_long_short_return_times(orc):
    """Sec. III.C: trajectories born near -80 and 20 a.u. return in t = [60, 90];
    the first is a long, the second a short trajectory (free motion from the
    first-order tunnel exit in the oracle's field)."""
    g = PAPER["n2_theta0_trajectories"]
    p = workloads.n2()
    w, E0, tau, N = orc.laser(p)
    T = 2 * math.pi / w
    t = np.linspace(-tau / 2, tau / 2, 200001)
    E, A = orc.field(p, t)
    X = integrate.cumulative_trapezoid(A, t, initial=0.0)
    ret = {}
    for name, tb in (("long", g["long_birth"]), ("short", g["short_birth"])):
        i0 = int(np.argmin(np.abs(t - tb)))
        x = -p["target"]["Ip"] / E[i0] + X[i0:] - X[i0] - A[i0] * (t[i0:] - t[i0])
        s = np.sign(x)
        idx = np.nonzero(s[1:] != s[:-1])[0]
        assert idx.size
        ret[name] = (t[i0 + idx[0] + 1], t[i0 + idx[0] + 1] - tb)
    lo, hi = g["return_window"]
    for name in ret:
        assert lo - 5 <= ret[name][0] <= hi + 5, ret
    assert ret["long"][1] > 0.65 * T > ret["short"][1]


# --------------------------------------------------------------- potential
@pytest.mark.parametrize("mk", [workloads.h2_softcore, workloads.n2])
def test_potential_derivatives_finite_difference(orc, mk):
    p = mk(35.0)
    th = math.radians(35.0)
    n = np.array([math.sin(th), 0.0, math.cos(th)])
    rng = np.random.default_rng(5)
    for q in rng.normal(0, 1.5, (6, 3)):
        V, g, H = orc.potential(p, n, q)
        h = 1e-5
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            Vp, gp, _ = orc.potential(p, n, q + e)
            Vm, gm, _ = orc.potential(p, n, q - e)
            assert abs((Vp - Vm) / (2 * h) - g[a]) < 1e-7 * max(1, abs(g[a]))
            assert np.max(np.abs((gp - gm) / (2 * h) - H[:, a])) < 1e-6 * max(1, np.abs(H).max())
        assert np.allclose(H, H.T)


def test_potential_reduces_to_eq7(orc):
    """eps^2 = 0 gives Eq. (7) with the Table I parameters exactly."""
    t1 = PAPER["table_I_model_potential"]["N2"]
    p = workloads.n2()
    for c in p["target"]["centers"]:
        c["eps2"] = 0.0
    n = np.array([0.0, 0.6, 0.8])
    for q in ([0.3, -0.2, 1.7], [2.0, 1.0, -0.5]):
        q = np.array(q)
        want = 0.0
        for s in (1, -1):
            r = np.linalg.norm(q - s * t1["R"] / 2 * n)
            want -= (t1["Zinf"] + (t1["Z0"] - t1["Zinf"]) * math.exp(-t1["alpha"] * r)) / r
        V, _, _ = orc.potential(p, n, q)
        assert abs(V - want) < 1e-13 * abs(want)


# ------------------------------------------------------------- recombination
def _psi0_and_overlap_grid(p, nax, pt, qt, L=9.0, h=0.15):
    """rho = int d^3x psi0(x) (p_z + i gamma (z - q_z)) <x|p,q> by the trapezoid rule."""
    g = p["gamma"]
    R = p["target"]["R"]
    x = np.arange(-L, L + h / 2, h)
    X, Y = np.meshgrid(x, x, indexing="ij")
    tot = 0.0 + 0.0j
    for z in x:
        psi = np.zeros_like(X)
        for (ctr, l, a, c) in p["target"]["gto"]:
            cen = (R / 2 if ctr == 0 else -R / 2) * np.asarray(nax)
            dx, dy, dz = X - cen[0], Y - cen[1], z - cen[2]
            r2 = dx * dx + dy * dy + dz * dz
            ang = 1.0 if l == 0 else (nax[0] * dx + nax[1] * dy + nax[2] * dz)
            psi += c * ang * np.exp(-a * r2)
        ddx, ddy, ddz = X - qt[0], Y - qt[1], z - qt[2]
        cs = (g / math.pi) ** 0.75 * np.exp(-0.5 * g * (ddx ** 2 + ddy ** 2 + ddz ** 2)
                                           + 1j * (pt[0] * ddx + pt[1] * ddy + pt[2] * ddz))
        tot += np.sum(psi * (pt[2] + 1j * g * ddz) * cs)
    return tot * h ** 3


@pytest.mark.parametrize("mol", ["H2", "N2"])
def test_recombination_closed_form_vs_position_quadrature(orc, mol):
    """The momentum-space Gaussian closed form equals the position-space
    integral <psi0| -i d/dz |p,q> evaluated by brute-force quadrature."""
    p = workloads.h2_softcore() if mol == "H2" else workloads.n2()
    cases = [((0.0, 0.0, 1.0), (0.3, -0.2, 1.1), (0.4, 0.1, -0.6)),
             ((math.sin(0.7), 0.0, math.cos(0.7)), (-0.5, 0.8, 1.9), (0.2, -0.3, 0.5)),
             ((0.0, math.sin(1.2), math.cos(1.2)), (1.2, 0.0, -2.4), (-0.8, 0.4, 1.3))]
    for nax, pt, qt in cases:
        want = _psi0_and_overlap_grid(p, nax, pt, qt)
        got = orc.recombination(p, nax, pt, qt)
        assert abs(got - want) < 1e-9 * max(abs(want), 1e-3), (nax, pt, qt, got, want)


def test_recombination_gamma_general(orc):
    p = workloads.n2()
    p["gamma"] = 0.6
    nax, pt, qt = (0.0, 0.0, 1.0), (0.5, -0.4, 0.9), (0.3, 0.2, -0.7)
    want = _psi0_and_overlap_grid(p, nax, pt, qt, L=11.0, h=0.15)
    got = orc.recombination(p, nax, pt, qt)
    assert abs(got - want) < 1e-9 * abs(want)


# ---------------------------------------------------------------- prefactor
@pytest.mark.parametrize("gam", [0.5, 1.0, 2.0])
def test_prefactor_matched_oscillator(orc, gam):
    """For a harmonic oscillator of frequency gamma the coherent state stays a
    coherent state, so |det R| = 1 and det R = exp(-3 i gamma t)."""
    for t in (0.3, 1.7, 4.0):
        c, s = math.cos(gam * t), math.sin(gam * t)
        M = np.block([[c * np.eye(3), s / gam * np.eye(3)], [-gam * s * np.eye(3), c * np.eye(3)]])
        d = orc.prefactor_det(M.ravel(), gam)
        assert abs(d - np.exp(-3j * gam * t)) < 1e-14


def test_prefactor_symplectic_lower_bound(orc):
    """|det R| >= 1 for any symplectic M (R is the average of a symplectic
    map and its Gaussian-conjugate); random symplectic M = exp(J S)."""
    from scipy.linalg import expm
    rng = np.random.default_rng(3)
    J = J6()
    for gam in (0.5, 1.0, 2.0):
        for _ in range(200):
            S = rng.normal(size=(6, 6))
            S = S + S.T
            M = expm(J @ S * 0.4)
            assert np.allclose(M.T @ J @ M, J, atol=1e-9)
            assert abs(orc.prefactor_det(M.ravel(), gam)) >= 1 - 1e-10


# ------------------------------------------------------------- free motion
def _volkov(orc, p, k0, kend, q0, p0):
    w, E0, tau, N = orc.laser(p)
    t0, t1 = orc.time(p, k0), orc.time(p, kend)
    A = lambda t: orc.field(p, t)[1]
    A0, A1 = A(t0), A(t1)
    IA, _ = integrate.quad(A, t0, t1, limit=400, epsabs=1e-14, epsrel=1e-14)
    IA2, _ = integrate.quad(lambda t: A(t) ** 2, t0, t1, limit=400, epsabs=1e-14, epsrel=1e-14)
    dt = t1 - t0
    c = p0[2] - A0
    pf = np.array([p0[0], p0[1], p0[2] + A1 - A0])
    qf = np.array([q0[0] + p0[0] * dt, q0[1] + p0[1] * dt, q0[2] + c * dt + IA])
    S = 0.5 * (p0[0] ** 2 + p0[1] ** 2 + c * c) * dt - 0.5 * IA2 + qf[2] * A1 - q0[2] * A0
    return qf, pf, S


def test_volkov_closed_form(orc):
    """V = 0: p = p0 + A(t) - A(t0), q and S from the closed-form integrals."""
    p = workloads.free_problem(workloads.n2(20.0))
    q0 = np.array([0.5, -0.3, -8.0])
    p0 = np.array([0.2, -0.1, 0.3])
    N = orc.n_steps(p)
    for k0 in (1000, 6000):
        _, fin = orc.trajectory(p, k0, q0, p0, (0, 0, 1), k_end=N, amplitudes=False)
        qf, pf, S = _volkov(orc, p, k0, N, q0, p0)
        assert np.max(np.abs(fin[0:3] - qf)) < 1e-8 * max(1, np.abs(qf).max())
        assert np.max(np.abs(fin[3:6] - pf)) < 1e-10
        assert abs(fin[42] - S) < 1e-8 * max(1.0, abs(S))


def test_volkov_rk4_order(orc):
    """The Volkov error of the RK4 action falls ~16x per halving of dt."""
    base = workloads.free_problem(workloads.n2(0.0))
    q0 = np.array([0.0, 0.0, -9.0])
    p0 = np.array([0.1, 0.0, 0.0])
    errs = []
    for dt, k0, k1 in ((4.0, 20, 120), (2.0, 40, 240), (1.0, 80, 480)):
        p = dict(base, dt=dt)
        _, fin = orc.trajectory(p, k0, q0, p0, (0, 0, 1), k_end=k1, amplitudes=False)
        qf, pf, S = _volkov(orc, p, k0, k1, q0, p0)
        errs.append(abs(fin[42] - S) + abs(fin[2] - qf[2]))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def test_free_monodromy(orc):
    """V = 0: M = [[I, (t-t0) I], [0, I]] exactly (RK4 is exact for it)."""
    p = workloads.free_problem(workloads.h2_softcore(0.0))
    N = orc.n_steps(p)
    k0 = 1234
    _, fin = orc.trajectory(p, k0, (0.1, 0.2, -7.0), (0.3, -0.2, 0.1), (0, 0, 1), amplitudes=False)
    tt = orc.time(p, N) - orc.time(p, k0)
    M = fin[6:42].reshape(6, 6)
    want = np.block([[np.eye(3), tt * np.eye(3)], [np.zeros((3, 3)), np.eye(3)]])
    assert np.max(np.abs(M - want)) < 1e-11 * tt


@pytest.mark.parametrize("gam", [0.5, 1.0, 2.0])
def test_free_prefactor_continuous_branch(orc, gam):
    """V = 0: C = (1 - i gamma tau/2)^{3/2} on the continuous branch; arg(det R)
    passes -pi at tau = 2 sqrt(3)/gamma without a sign flip of C."""
    p = workloads.free_problem(workloads.h2_softcore(0.0))
    p["gamma"] = gam
    k0 = 500
    for steps in (10, 34, 35, 60, 200, 1500):
        _, fin = orc.trajectory(p, k0, (0, 0, -5.0), (0.2, 0.1, 0.0), (0, 0, 1), k_end=k0 + steps,
                                amplitudes=False)
        tau = orc.time(p, k0 + steps) - orc.time(p, k0)
        want = np.exp(1.5 * np.log(1 - 0.5j * gam * tau))
        got = fin[43] + 1j * fin[44]
        assert abs(got - want) < 1e-12 * abs(want), (steps, got, want)
        assert fin[45] == 0


# ---------------------------------------------------------------- invariants
def _live_ics(orc, p, seed, count, first=0):
    s = orc.sample(p, seed, first, 4000)
    idx = np.nonzero(s["w"] > 0)[0][:count]
    return [(int(s["k0"][i]), s["q0"][i], s["p0"][i], s["nax"][i], s["w"][i]) for i in idx]


def test_monodromy_symplectic_with_potential(orc):
    """det M = 1 and M^T J M = J up to the RK4 truncation (Liouville)."""
    p = workloads.n2(30.0)
    J = J6()
    for (k0, q0, p0, n, w) in _live_ics(orc, p, 1002, 6):
        _, fin = orc.trajectory(p, k0, q0, p0, n, w, amplitudes=False)
        M = fin[6:42].reshape(6, 6)
        nm = np.linalg.norm(M, 2)
        assert abs(np.linalg.det(M) - 1) < 1e-7 * nm ** 2
        assert np.max(np.abs(M.T @ J @ M - J)) < 1e-7 * nm ** 2
        R = 0.5 * (M[:3, :3] + M[3:, 3:] - 1j * p["gamma"] * M[:3, 3:] + 1j / p["gamma"] * M[3:, :3])
        assert abs(np.linalg.det(R)) >= 1 - 1e-6


def test_action_variation_is_endpoint_momentum(orc):
    """Hamilton's principal function: along solutions the first variation of
    the action is dS = p_T . dq_T - p_0 . dq_0 (the Euler-Lagrange terms
    vanish).  Two trajectories started at q0 +/- delta e in the full potential
    and laser, same p0: their action difference equals the endpoint terms to
    O(delta^2) and the RK4 truncation.  Pins the potential and field terms of
    the action's integrand (the Volkov pins have V = 0)."""
    p = workloads.n2(30.0)
    ics = _live_ics(orc, p, 1002, 2)
    N = orc.n_steps(p)
    d = 1e-4
    for (k0, q0, p0, n, w) in ics:
        kend = min(N, k0 + 2000)
        for e in np.eye(3):
            _, fp = orc.trajectory(p, k0, q0 + d * e, p0, n, k_end=kend, amplitudes=False)
            _, fm = orc.trajectory(p, k0, q0 - d * e, p0, n, k_end=kend, amplitudes=False)
            dS = fp[42] - fm[42]
            want = 0.5 * (fp[3:6] + fm[3:6]) @ (fp[0:3] - fm[0:3]) - p0 @ (2 * d * e)
            assert abs(dS - want) <= 1e-6 * abs(want) + 1e-12, (k0, e, dS, want)


def test_energy_conserved_laser_off(orc):
    """E = 0: H = p^2/2 + V is conserved; drift ~dt^4."""
    base = workloads.laser_off(workloads.n2(25.0))
    th = math.radians(25.0)
    n = np.array([math.sin(th), 0, math.cos(th)])
    q0 = np.array([1.2, -0.4, 2.5])
    p0 = np.array([0.3, 0.5, -0.9])
    drifts = []
    for dt, steps in ((0.04, 500), (0.02, 1000), (0.01, 2000)):
        p = dict(base, dt=dt)
        _, fin = orc.trajectory(p, 0, q0, p0, n, k_end=steps, amplitudes=False)
        H0 = 0.5 * p0 @ p0 + orc.potential(p, n, q0)[0]
        H1 = 0.5 * fin[3:6] @ fin[3:6] + orc.potential(p, n, fin[0:3])[0]
        drifts.append(abs(H1 - H0))
    assert drifts[0] < 1e-4
    assert drifts[0] / drifts[1] > 10 and drifts[1] / drifts[2] > 10, drifts


def test_monodromy_equals_finite_difference_jacobian(orc):
    """M is the Jacobian of the discrete RK4 map: central differences of the
    final (q, p) with respect to (q0, p0)."""
    p = workloads.n2(40.0)
    th = math.radians(40.0)
    n = np.array([math.sin(th), 0, math.cos(th)])
    k0, q0, p0 = 5000, np.array([0.4, 0.2, -6.0]), np.array([0.1, -0.2, 0.05])
    kend = k0 + 800
    _, fin = orc.trajectory(p, k0, q0, p0, n, k_end=kend, amplitudes=False)
    M = fin[6:42].reshape(6, 6)
    h = 1e-6
    x0 = np.concatenate([q0, p0])
    for c in range(6):
        e = np.zeros(6)
        e[c] = h
        _, fp = orc.trajectory(p, k0, (x0 + e)[:3], (x0 + e)[3:], n, k_end=kend, amplitudes=False)
        _, fm = orc.trajectory(p, k0, (x0 - e)[:3], (x0 - e)[3:], n, k_end=kend, amplitudes=False)
        col = (fp[0:6] - fm[0:6]) / (2 * h)
        assert np.max(np.abs(col - M[:, c])) < 1e-6 * max(1.0, np.abs(M).max())


# ---------------------------------------------------------------- symmetries
def test_axial_symmetry_theta0(orc):
    """theta = 0: rotating p_perp by pi about the field axis leaves every
    trajectory's amplitude unchanged."""
    p = workloads.n2(0.0)
    for (k0, q0, p0, n, w) in _live_ics(orc, p, 1002, 5):
        a1, _ = orc.trajectory(p, k0, q0, p0, n, w)
        a2, _ = orc.trajectory(p, k0, q0 * [-1, -1, 1], p0 * [-1, -1, 1], n, w)
        assert np.max(np.abs(a1 - a2)) <= 1e-9 * np.max(np.abs(a1))


def test_mirror_theta_pi_minus_theta(orc):
    """theta and 180 - theta with p_x mirrored give the same amplitudes
    (homonuclear target, mirror x -> -x)."""
    pa, pb = workloads.n2(30.0), workloads.n2(150.0)
    ta, tb = math.radians(30.0), math.radians(150.0)
    na = np.array([math.sin(ta), 0, math.cos(ta)])
    nb = np.array([math.sin(tb), 0, math.cos(tb)])
    for (k0, q0, p0, n, w) in _live_ics(orc, pa, 1002, 4):
        a1, _ = orc.trajectory(pa, k0, q0, p0, na, w)
        a2, _ = orc.trajectory(pb, k0, q0 * [-1, 1, 1], p0 * [-1, 1, 1], nb, w)
        assert np.max(np.abs(a1 - a2)) <= 1e-9 * np.max(np.abs(a1))


def test_axis_inversion_invariance(orc):
    """n -> -n swaps the two identical centres: V and the gerade orbital are
    unchanged, so are the amplitudes."""
    p = workloads.n2(50.0)
    th = math.radians(50.0)
    n = np.array([math.sin(th), 0, math.cos(th)])
    for (k0, q0, p0, _, w) in _live_ics(orc, p, 7, 3):
        a1, _ = orc.trajectory(p, k0, q0, p0, n, w)
        a2, _ = orc.trajectory(p, k0, q0, p0, -n, w)
        assert np.max(np.abs(a1 - a2)) <= 1e-9 * np.max(np.abs(a1))


# ------------------------------------------------------------- convergence
def test_dt_convergence_fourth_order(orc):
    """Brute-force dt convergence of the dipole of a tiny ensemble."""
    base = workloads.h2_softcore(0.0)
    ics = _live_ics(orc, base, 1001, 6)
    vs = []
    for f in (1, 2, 4):
        p = dict(base, dt=base["dt"] / f, n_steps=orc.n_steps(base) * f)
        N = orc.n_steps(p)
        acc = np.zeros(N + 1, dtype=complex)
        for (k0, q0, p0, n, w) in ics:
            a, _ = orc.trajectory(p, k0 * f, q0, p0, n, w)
            acc += a
        vs.append(acc[::f].real)
    r = np.linalg.norm(vs[0] - vs[1]) / np.linalg.norm(vs[1] - vs[2])
    assert 10 < r < 24, r


def test_linearity_of_ensemble_sum(orc):
    p = workloads.h2_softcore(0.0)
    a, ls_a, nl_a = orc.run(p, 1001, 0, 120, nthreads=2)
    b, ls_b, nl_b = orc.run(p, 1001, 120, 80, nthreads=3)
    c, ls_c, nl_c = orc.run(p, 1001, 0, 200, nthreads=4)
    assert np.max(np.abs(a + b - c)) < 1e-12 * np.max(np.abs(c))
    assert ls_a + ls_b == ls_c and nl_a + nl_b == nl_c


def test_free_monodromy_max_entry(orc):
    """V = 0: the largest monodromy entry along a trajectory is max(1, t_N - t0)
    (M = [[I, (t - t0) I], [0, I]]), for every trajectory of a run."""
    p = workloads.free_problem(workloads.h2_softcore(0.0))
    N = orc.n_steps(p)
    r = orc.run_ensemble(p, 1001, 0, 300, m_regular=1e4, nthreads=4)
    s = orc.sample(p, 1001, 0, 300)
    live = s["w"] > 0
    assert live.sum() > 50
    tN = orc.time(p, N)
    want = np.array([max(1.0, tN - orc.time(p, int(k))) for k in s["k0"]])
    got = r["finals"][:, orc.F_MMAX]
    assert np.all(np.abs(got[live] - want[live]) <= 1e-11 * want[live])
    assert np.all(r["finals"][~live] == 0.0)


def test_split_ensemble_sum(orc):
    """The split run on an N2 sample with chaotic trajectories: the full sum
    equals the plain run; the regular part plus the chaotic trajectories'
    amplitudes, each propagated alone, gives the full sum; the running maximum
    bounds the final monodromy; thresholds at infinity and below 1 select
    everything and nothing (M starts at the identity)."""
    p = workloads.n2(0.0)
    n, seed, nt = 2000, 1002, 8
    r = orc.run_ensemble(p, seed, 0, n, m_regular=1e4, nthreads=nt)
    acc, ls, nl = orc.run(p, seed, 0, n, nthreads=nt)
    assert np.array_equal(r["accum_all"], acc)
    assert (r["live_steps"], r["n_live"]) == (ls, nl)
    s = orc.sample(p, seed, 0, n)
    fin = r["finals"]
    live = s["w"] > 0
    mmax = fin[:, orc.F_MMAX]
    chaotic = np.nonzero(live & (mmax > 1e4))[0]
    assert 0 < len(chaotic) < 0.05 * live.sum()
    assert np.all(mmax[live] >= np.max(np.abs(fin[live, 6:42]), axis=1))
    assert np.all(mmax[live] >= 1.0)
    extra = np.zeros_like(acc)
    for i in chaotic:
        a, _ = orc.trajectory(p, int(s["k0"][i]), s["q0"][i], s["p0"][i], s["nax"][i], w=s["w"][i])
        extra += a.real
    scale = np.max(np.abs(acc))
    assert np.max(np.abs(r["accum_regular"] + extra - acc)) <= 1e-12 * scale
    r_all = orc.run_ensemble(p, seed, 0, 300, m_regular=np.inf, nthreads=nt, finals=False)
    assert np.array_equal(r_all["accum_regular"], r_all["accum_all"])
    r_none = orc.run_ensemble(p, seed, 0, 300, m_regular=0.5, nthreads=nt, finals=False)
    assert np.all(r_none["accum_regular"] == 0.0) and np.any(r_none["accum_all"] != 0.0)


# ---------------------------------------------------------------- spectrum
def test_spectrum_equals_fft(orc):
    """On the FFT grid the windowed transform is a library FFT."""
    rng = np.random.default_rng(2)
    n, dt, t_first = 1024, 0.1, -51.15
    tau_h = 45.0
    v = rng.normal(size=n)
    t = t_first + dt * np.arange(n)
    wh = np.where(np.abs(t) <= tau_h, 0.5 * (1 + np.cos(np.pi * t / tau_h)), 0.0)
    m = np.arange(0, 200)
    om = 2 * np.pi * m / (n * dt)
    V, Y = orc.spectrum(v, t_first, dt, tau_h, om)
    want = dt * np.exp(1j * om * t_first) * n * np.fft.ifft(v * wh)[m]
    assert np.max(np.abs(V - want)) < 1e-11 * np.max(np.abs(want))
    assert np.allclose(Y, om ** 2 * np.abs(want) ** 2, rtol=1e-10, atol=0)


def test_spectrum_of_windowed_cosine(orc):
    """A pure harmonic peaks at its own frequency with the Hanning main lobe."""
    dt, tau_h = 0.05, 300.0
    t = np.arange(-6000, 6001) * dt
    w0 = 0.9
    om = np.linspace(0.5, 1.3, 801)
    V, Y = orc.spectrum(np.cos(w0 * t), t[0], dt, tau_h, om)
    assert abs(om[np.argmax(np.abs(V))] - w0) < 1e-3
    # continuous transform of cos(w0 t) W_H at w0: tau_h/2 (+ negligible image term)
    assert abs(np.abs(V).max() - tau_h / 2) < 1e-3 * tau_h


# ----------------------------------------------------------------- sampler
def test_sampler_distributions(orc):
    p = workloads.n2(0.0)
    w_, E0, tau, N = orc.laser(p)
    n = 200000
    s = orc.sample(p, 99, 0, n)
    # p_perp: N(0, sigma^2) per component, p_par = 0
    for c in (0, 1):
        x = s["p0"][:, c] / p["sigma_perp"]
        assert stats.kstest(x, "norm").pvalue > 1e-3
    assert np.all(s["p0"][:, 2] == 0)
    # birth step: uniform on 0..N-1
    assert s["k0"].min() >= 0 and s["k0"].max() <= N - 1
    hist = np.bincount(s["k0"] * 20 // N, minlength=20)
    assert stats.chisquare(hist).pvalue > 1e-3
    # weights: positive only above the cut, w(F0) = 1, increasing in |E|
    live = s["w"] > 0
    assert np.all(s["w"][live] >= p["w_cut"])
    assert 0.35 < live.mean() < 0.65
    E, _ = orc.field(p, -tau / 2 + s["k0"][live] * p["dt"])
    order = np.argsort(np.abs(E))
    assert np.all(np.diff(s["w"][live][order]) >= -1e-15)
    assert s["w"].max() <= 1.0 + 1e-12
    # tunnel exit on the field axis, opposite to the force -E: q0 . E < 0
    assert np.all(s["q0"][live, 2] * E < 0) and np.all(s["q0"][:, :2] == 0)


def test_sampler_cos4_axis(orc):
    p = workloads.n2(align=workloads.cos2m(2))
    s = orc.sample(p, 123, 0, 100000)
    cb = s["nax"][:, 2]
    assert np.allclose(np.linalg.norm(s["nax"], axis=1), 1.0)
    # density ~ cos^4(beta) sin(beta): CDF of u = cos(beta) is (u^5 + 1)/2
    assert stats.kstest(cb, lambda u: (u ** 5 + 1) / 2).pvalue > 1e-3
    al = np.arctan2(s["nax"][:, 1], s["nax"][:, 0]) % (2 * np.pi)
    assert stats.kstest(al / (2 * np.pi), "uniform").pvalue > 1e-3
    iso = orc.sample(workloads.n2(align=workloads.cos2m(0)), 5, 0, 100000)
    assert stats.kstest(iso["nax"][:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3


def test_philox_bits(orc):
    """Output bits balanced and a one-bit counter change flips about half the
    output bits (avalanche) for the counter-based generator."""
    outs = np.array([orc.philox([i, 0, 7, 0], [1234, 5678]) for i in range(20000)], dtype=np.uint64)
    bits = np.unpackbits(outs.astype(">u4").view(np.uint8)).reshape(-1, 128).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.02)
    flips = []
    for i in range(300):
        a = np.array(orc.philox([i, 9, 0, 0], [1, 2]), dtype=np.uint64)
        b = np.array(orc.philox([i ^ (1 << (i % 32)), 9, 0, 0], [1, 2]), dtype=np.uint64)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    assert abs(np.mean(flips) - 64) < 3
    assert orc.philox([0, 0, 0, 0], [0, 0]) != orc.philox([0, 0, 0, 0], [1, 0])


def test_emission_frequency_is_kinetic_plus_ip(orc):
    """No-depletion dipole (Sec. II.A): the ground state turns as e^{+i Ip t}
    and a continuum packet of energy E as e^{-i E t}, so their overlap
    oscillates at E + Ip.  A free electron (V = 0, laser off) in a wide
    coherent state (gamma = 0.004, nearly a plane wave) crossing a compact s
    orbital: the amplitude's spectrum peaks at p^2/2 + Ip."""
    p = workloads.laser_off(workloads.free_problem(workloads.n2(0.0)))
    p["target"]["R"] = 0.0
    p["target"]["gto"] = [(0, 0, 1e4, 1.0)]
    p["gamma"] = 0.004
    Ip = p["target"]["Ip"]
    dt = p["dt"]
    for pz in (1.0, 1.5):
        k0, z0 = 10, -110.0
        kend = k0 + int(round(-2 * z0 / pz / dt))
        a, _ = orc.trajectory(p, k0, (0, 0, z0), (0, 0, pz), (0, 0, 1), 1.0, k_end=kend)
        seg = a[k0:kend + 1]
        nfft = 1 << 18
        spec = np.abs(np.fft.fft(seg, nfft))          # e^{-i w t} kernel: peak at the turning rate
        om = 2 * np.pi * np.fft.fftfreq(nfft, dt)
        peak = -om[np.argmax(spec)]
        want = 0.5 * pz * pz + Ip
        assert abs(peak - want) < 0.01 * want, (pz, peak, want)


def _exact_saddle(p, orc, t0, kperp2=0.0):
    """Exact complex saddle point of Eq. (2) for k = (k_perp, 0) and the full A(t)
    continued to complex time (Newton), the tunnelling action Im S_down^0 and
    the tunnel exit Re int_{ts}^{t0} A along the vertical path."""
    w, E0, tau, N = orc.laser(p)
    Ip = p["target"]["Ip"]
    cep = p["laser"]["cep"]
    A = lambda t: -(E0 / w) * np.cos(np.pi * t / tau) ** 2 * np.sin(w * t + cep)
    Ef = lambda t: (E0 * np.cos(np.pi * t / tau) ** 2 * np.cos(w * t + cep)
                    - (E0 * np.pi / (w * tau)) * np.sin(2 * np.pi * t / tau) * np.sin(w * t + cep))
    F = Ef(t0)
    A0 = A(t0)
    target = -1j * np.sign(F) * math.sqrt(2 * Ip + kperp2)
    ts = t0 + 1j * math.sqrt(2 * Ip + kperp2) / abs(F)
    for _ in range(60):
        ts = ts + (A(ts) - A0 - target) / Ef(ts)
    xs, ws = np.polynomial.legendre.leggauss(64)
    y = ts.imag
    s = 0.5 * (xs + 1) * y
    wq = 0.5 * y * ws
    path = t0 + 1j * s
    int_A = -1j * np.sum(wq * A(path))                     # int_{ts}^{t0} A
    int_K = -1j * np.sum(wq * (kperp2 + (A(path) - A0) ** 2) / 2)
    return (Ip * ts - int_K).imag, int_A.real


def test_tunnel_exit_and_weight_against_exact_saddle_point(orc):
    """The sampler's first-order tunnel exit and tunnelling exponent converge
    to the exact saddle point of Eq. (2) as the Keldysh parameter falls
    (quasi-static limit, errors ~ gamma_K^2), near the field crests.  The
    weight is the p = 0 amplitude; the exit uses the sampled p_perp."""
    errs = {}
    for lam in (4000.0, 12000.0):
        p = workloads.n2(0.0, laser=dict(workloads.N2_LASER, lambda_nm=lam))
        w, E0, tau, N = orc.laser(p)
        Ip = p["target"]["Ip"]
        kap = math.sqrt(2 * Ip)
        pw = 0.5 * (2 / kap - 1)
        ims_peak, _ = _exact_saddle(p, orc, 0.0)
        s = orc.sample(p, 3, 0, 3000)
        e_exp, e_q = [], []
        for i in np.nonzero(s["w"] > 0)[0]:
            t0 = orc.time(p, s["k0"][i])
            E, _ = orc.field(p, t0)
            if abs(E) < 0.8 * E0:
                continue
            ims, _ = _exact_saddle(p, orc, t0)
            _, qx = _exact_saddle(p, orc, t0, float(s["p0"][i, 0] ** 2 + s["p0"][i, 1] ** 2))
            expo = math.log(s["w"][i]) - pw * math.log(E0 / abs(E))   # exponential part of w
            if abs(ims - ims_peak) > 1e-6:
                e_exp.append(abs(expo + (ims - ims_peak)) / abs(ims - ims_peak))
            e_q.append(abs(s["q0"][i, 2] - qx) / abs(qx))
        assert len(e_q) > 20
        errs[lam] = (max(e_exp), max(e_q))
    assert errs[12000.0][0] < 0.005 and errs[12000.0][1] < 0.01, errs
    assert errs[4000.0][0] / errs[12000.0][0] > 5 and errs[4000.0][1] / errs[12000.0][1] > 5, errs


def test_prefactor_cap_truncates_contributions(orc):
    """With a prefactor cap, a trajectory's amplitudes are the uncapped ones up
    to the first step with |C_k| > c_max and zero from there on; a cap above
    every |C_k| changes nothing."""
    p = workloads.n2(0.0)
    ics = _live_ics(orc, p, 1002, 12)
    hit = 0
    for (k0, q0, p0, n, w) in ics:
        a, _, c = orc.trajectory(p, k0, q0, p0, n, w, prefactors=True)
        cmax = 30.0
        capped = dict(p, c_max=cmax)
        ac, _ = orc.trajectory(capped, k0, q0, p0, n, w)
        over = np.nonzero(np.abs(c[k0:]) > cmax)[0]
        kc = k0 + over[0] if over.size else len(a)
        hit += over.size > 0
        assert np.array_equal(ac[:kc], a[:kc])
        assert np.all(ac[kc:] == 0)
        big = dict(p, c_max=10 * np.abs(c).max() + 1)
        ab, _ = orc.trajectory(big, k0, q0, p0, n, w)
        assert np.array_equal(ab, a)
    assert hit > 0


def test_averaging_quadrature_integrates_the_isotropic_density():
    """The 10 fixed alignments of the standard average integrate any
    polynomial of cos(theta) up to degree 19 over the isotropic density
    (1/2) sin(theta) d(theta) on [0, pi] exactly (even polynomials, by the
    homonuclear symmetry), and the joint problem samples the sphere uniformly."""
    import workloads as W
    av = W.workload_averaging("H2", 10)
    probs, wts = av["standard"]
    assert abs(sum(wts) - 1.0) < 1e-15
    xs = [math.cos(p["align"]["theta"]) for p in probs]
    for k in range(0, 20, 2):
        exact = 1.0 / (k + 1)  # (1/2) int_{-1}^{1} x^k dx
        assert abs(sum(w * x ** k for w, x in zip(wts, xs)) - exact) < 1e-14
    assert av["joint"]["align"] == {"kind": "cos2m", "theta": 0.0, "phi": 0.0, "m": 0}


# ------------------------------------------------- spectrum on the FFT grid
def _fft_case(n=1000, seed=3):
    rng = np.random.default_rng(seed)
    dt, t_first = 0.1, -0.5 * (n - 1) * 0.1
    t = t_first + np.arange(n) * dt
    v = rng.normal(size=n) * 0.1 + np.cos(0.057 * 7 * t) + 0.3 * np.sin(0.057 * 13 * t + 0.4)
    return v, t_first, dt, 0.5 * n * dt


def test_fft_spectrum_equals_direct_transform(orc):
    """Eq. 3 on the FFT grid equals the direct sum (itself pinned by closed
    forms) at the same frequencies, for bins across the whole grid."""
    v, t_first, dt, tau_H = _fft_case()
    w, V, Y, ph = orc.spectrum_fft(v, t_first, dt, tau_H)
    L = 2 * (w.size - 1)
    assert L == 1 << orc.fft_log2_len(v.size) and L >= 8 * v.size
    j = np.array([0, 1, 2, 17, 333, 1234, L // 4, L // 2 - 1, L // 2])
    Vd, Yd = orc.spectrum(v, t_first, dt, tau_H, w[j])
    assert np.max(np.abs(V[j] - Vd)) < 1e-12 * np.max(np.abs(Vd))
    assert np.allclose(Y[j], Yd, rtol=1e-10, atol=1e-14 * Yd.max())
    # A = -i w V: |A|^2 is the yield, its phase is arg V - pi/2 (w > 0)
    sel = j[1:]
    d = np.angle(np.exp(1j * (ph[sel] - np.angle(V[sel]) + np.pi / 2)))
    assert np.max(np.abs(d)) < 1e-12


def test_fft_spectrum_parseval_and_padding(orc):
    """Parseval for the real windowed signal, and twice the padding puts the
    same values on every second bin (the time origin t_first is kept)."""
    v, t_first, dt, tau_H = _fft_case(777, 5)
    w, V, Y, _ = orc.spectrum_fft(v, t_first, dt, tau_H)
    L = 2 * (w.size - 1)
    t = t_first + np.arange(v.size) * dt
    x = v * np.where(np.abs(t) <= tau_H, 0.5 * (1 + np.cos(np.pi * t / tau_H)), 0.0)
    X2 = np.abs(V / dt) ** 2
    assert abs((X2[0] + 2 * X2[1:-1].sum() + X2[-1]) / L - np.sum(x * x)) < 1e-10 * np.sum(x * x)
    w2, V2, _, _ = orc.spectrum_fft(v, t_first, dt, tau_H, orc.fft_log2_len(v.size) + 1)
    assert np.allclose(w2[::2], w) and np.max(np.abs(V2[::2] - V)) < 1e-12 * np.abs(V).max()


def test_acceleration_is_the_derivative_of_the_windowed_dipole(orc):
    """The acceleration on the step grid from the zero-padded spectrum equals
    the closed-form derivative of a windowed tone, W_H' cos(w0 t) -
    W_H w0 sin(w0 t), to the resolution of the sampling (the window's second
    derivative jumps at +-tau_H), and halving dt shrinks the error (5.3e-7 to
    3.5e-7 here)."""
    errs = []
    for n, dt in ((3311, 0.1), (6621, 0.05)):
        t_first, tau_H, w0 = -0.5 * (n - 1) * dt, 0.25 * (n - 1) * dt, 0.057 * 9
        t = t_first + np.arange(n) * dt
        inside = np.abs(t) <= tau_H
        wh = np.where(inside, 0.5 * (1 + np.cos(np.pi * t / tau_H)), 0.0)
        dwh = np.where(inside, -0.5 * np.pi / tau_H * np.sin(np.pi * t / tau_H), 0.0)
        exact = dwh * np.cos(w0 * t) - wh * w0 * np.sin(w0 * t)
        a = orc.acceleration_fft(np.cos(w0 * t), t_first, dt, tau_H)
        errs.append(np.max(np.abs(a - exact)) / np.max(np.abs(exact)))
    assert errs[0] < 1e-5 and errs[1] < 0.8 * errs[0], errs

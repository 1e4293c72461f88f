"""Pins of the oracle's exact SFA ionisation step (Sec. II.A, Eq. 1-2): the
saddle point, the tunnel exit, the tunnelling action and the ionisation
matrix element, each checked against something other than the oracle's own
formulas: closed forms for a monochromatic field, the adiabatic (first-order)
limit, analyticity of the continued field, one-dimensional quadrature of the
Gaussian integrals, and the inversion symmetry of a gerade orbital."""
import cmath
import math

import numpy as np
import pytest

import workloads as W


def saddle(p):
    return W.with_changes(p, ionization="saddle")


def test_continued_field_is_analytic_and_minus_dA_dt(orc):
    """E(t) = -dA/dt at complex t: the derivative taken along the imaginary
    direction (Cauchy-Riemann) equals the one along the real direction."""
    p = W.n2(0.0)
    h = 1e-4
    for tr, ti in [(0.0, 10.0), (-40.0, 17.0), (55.0, 30.0)]:
        A_r1, _ = orc.field_complex(p, tr + h, ti)
        A_r0, _ = orc.field_complex(p, tr - h, ti)
        A_i1, _ = orc.field_complex(p, tr, ti + h)
        A_i0, _ = orc.field_complex(p, tr, ti - h)
        _, E = orc.field_complex(p, tr, ti)
        d_real = (A_r1 - A_r0) / (2 * h)
        d_imag = (A_i1 - A_i0) / (2j * h)
        assert abs(d_real - d_imag) < 1e-8 * max(1.0, abs(d_real))
        assert abs(d_real + E) < 1e-8 * max(1.0, abs(E))
    # on the real axis the continuation is the pulse itself
    for t in [-100.0, 3.0, 250.0]:
        A, E = orc.field_complex(p, t, 0.0)
        E0, A0 = orc.field(p, t)
        assert abs(A - A0) < 1e-15 and abs(E - E0) < 1e-15


def test_saddle_point_solves_eq2(orc):
    p = saddle(W.n2(30.0))
    Ip = p["target"]["Ip"]
    rng = np.random.default_rng(5)
    for _ in range(20):
        t0 = rng.uniform(-200, 200)
        kp = rng.normal(0, 0.3, 2)
        r = orc.sfa_step(p, t0, kp, (0.5, 0.0, math.sqrt(0.75)))
        if r is None:
            continue
        _, A0 = orc.field(p, t0)
        As, _ = orc.field_complex(p, t0, r["tt"])
        kz_s = r["kz"] + As - A0
        assert abs(kp @ kp + kz_s ** 2 + 2 * Ip) < 1e-11
        assert r["tt"] > 0
        # no smaller root: h(s) = |Im A(t0 + i s)| stays below kappa0 before t_t
        E0, _ = orc.field(p, t0)
        kap0 = math.sqrt(2 * Ip + kp @ kp)
        for s in np.linspace(0, r["tt"], 50)[1:-1]:
            As, _ = orc.field_complex(p, t0, s)
            assert -math.copysign(1, E0) * As.imag < kap0


def monochromatic_reference(E0, w, phi0, Ip, kp2):
    """Closed forms for A(t) = -(E0/w) sin(w t + phi) with phi0 = w t0 + phi:
    t_t from (E0/w)|cos phi0| sinh(w t_t) = kappa0, k_z = A(t0) - Re A(t_s),
    q0 = Re int_{t_s}^{t0} A dt, and S = I_p t_s - int_{t_s}^{t0} kappa^2/2 dt
    with the elementary integrals of cosh and sinh."""
    kap0 = math.sqrt(2 * Ip + kp2)
    a0 = E0 / w
    c, s = math.cos(phi0), math.sin(phi0)
    tt = math.asinh(kap0 / (a0 * abs(c))) / w
    C = math.cosh(w * tt)
    kz = -a0 * s * (1 - C)
    q0 = -(a0 / w) * c * (C - 1)
    sh, sh2 = math.sinh(w * tt), math.sinh(2 * w * tt)
    int_ch2 = tt / 2 + sh2 / (4 * w)
    int_sh2 = -tt / 2 + sh2 / (4 * w)
    int_re = s * s * (int_ch2 - 2 * C * sh / w + C * C * tt) - c * c * int_sh2
    ImS = (Ip + kp2 / 2) * tt + 0.5 * a0 * a0 * int_re
    int_im = 2 * s * c * (sh * sh / (2 * w) - C * (C - 1) / w)
    ReS_minus = -0.5 * a0 * a0 * int_im
    return tt, kz, q0, ImS, ReS_minus


@pytest.mark.parametrize("t0,kp", [(0.0, (0.0, 0.0)), (12.0, (0.2, -0.1)),
                                   (-25.0, (0.05, 0.3)), (40.0, (0.0, 0.15))])
def test_monochromatic_closed_forms(orc, t0, kp):
    """A 60,000-cycle pulse is monochromatic near its centre: its envelope
    changes the results by below 1e-8 relative (the differences fall as the
    inverse square of the cycle count)."""
    p = saddle(W.n2(0.0, laser=dict(W.N2_LASER, n_cycles=60000.0, cep=0.3)))
    w, E0, tau, N = orc.laser(p)
    Ip = p["target"]["Ip"]
    r = orc.sfa_step(p, t0, kp, (0, 0, 1))
    kp2 = kp[0] ** 2 + kp[1] ** 2
    tt, kz, q0, ImS, ReSm = monochromatic_reference(E0, w, w * t0 + 0.3, Ip, kp2)
    assert r["tt"] == pytest.approx(tt, rel=1e-6)
    assert r["kz"] == pytest.approx(kz, abs=1e-6)
    assert r["q0z"] == pytest.approx(q0, rel=1e-6)
    assert r["S"].imag == pytest.approx(ImS, rel=1e-6)
    assert r["S"].real - Ip * t0 == pytest.approx(ReSm, abs=1e-6)


def test_adiabatic_limit_is_the_first_order_step(orc):
    """At a field maximum and vanishing Keldysh parameter the saddle point
    tends to the first-order expansion: t_t -> kappa0/E, q0 -> -(I_p +
    k_perp^2/2)/E, Im S -> kappa0^3/(3E), k_z -> 0; the corrections are
    O(gamma_K^2)."""
    errs, phase = [], []
    for lam in (4000.0, 8000.0, 16000.0):
        p = saddle(W.n2(0.0, laser=dict(W.N2_LASER, lambda_nm=lam, n_cycles=8.0)))
        w, E0, tau, N = orc.laser(p)
        Ip = p["target"]["Ip"]
        kp = (0.1, 0.0)
        r = orc.sfa_step(p, 0.0, kp, (0, 0, 1))
        E, _ = orc.field(p, 0.0)
        kap0 = math.sqrt(2 * Ip + 0.01)
        gam = w * math.sqrt(2 * Ip) / E0
        e = max(abs(r["tt"] / (kap0 / E) - 1), abs(r["q0z"] / (-(Ip + 0.005) / E) - 1),
                abs(r["S"].imag / (kap0 ** 3 / (3 * E)) - 1))
        assert abs(r["kz"]) < 1e-12
        assert e < 0.5 * gam * gam
        errs.append(e)
        # off the peak (laser phase 0.15) Re S - I_p t0, zero in the first-order
        # reading, vanishes linearly in the laser frequency
        r = orc.sfa_step(p, 0.15 / w, kp, (0, 0, 1))
        phase.append(abs(r["S"].real - Ip * 0.15 / w))
    assert errs[0] > errs[1] > errs[2]  # shrinks with gamma_K^2
    assert phase[0] / phase[1] == pytest.approx(2.0, rel=0.1)
    assert phase[1] / phase[2] == pytest.approx(2.0, rel=0.1)


def _gauss_moments_1d(a, center, kc, order):
    """int x^order e^{-i kc x} e^{-a (x - center)^2} dx by fine quadrature on
    a real grid (kc complex: the exponential growth of e^{-i kc x} is beaten
    by the Gaussian)."""
    span = 12.0 / math.sqrt(a) + abs(kc.imag) / a
    x = np.linspace(center - span, center + span + 2 * abs(kc.imag) / a, 40001)
    f = x ** order * np.exp(-1j * kc * x - a * (x - center) ** 2)
    return np.trapezoid(f, x)


@pytest.mark.parametrize("mol,theta", [("H2", 0.0), ("N2", 0.0), ("N2", 50.0)])
def test_ionisation_matrix_element_by_quadrature(orc, mol, theta):
    """m sqrt(E kappa_z)/E = (2 pi)^{-3/2} int e^{-i kappa.x} z psi_0(x) d^3x
    at the complex saddle-point momentum, each primitive's 3D integral taken
    as products of 1D quadratures."""
    base = W.h2_softcore(theta) if mol == "H2" else W.n2(theta)
    p = saddle(base)
    th = math.radians(theta)
    n = np.array([math.sin(th), 0.0, math.cos(th)])
    t0, kp = 8.0, (0.15, -0.1)
    r = orc.sfa_step(p, t0, kp, n)
    _, A0 = orc.field(p, t0)
    As, Es = orc.field_complex(p, t0, r["tt"])
    kap = np.array([kp[0], kp[1], r["kz"] + As - A0], dtype=complex)
    me_oracle = r["m"] * cmath.sqrt(Es * kap[2]) / Es
    R = p["target"]["R"]
    total = 0j
    for ctr, l, a, c in p["target"]["gto"]:
        Rc = (1.0 if ctr == 0 else -1.0) * 0.5 * R * n
        m0 = [_gauss_moments_1d(a, Rc[j], kap[j], 0) for j in range(3)]
        m1 = [_gauss_moments_1d(a, Rc[j], kap[j], 1) for j in range(3)]
        m2z = _gauss_moments_1d(a, Rc[2], kap[2], 2)
        if l == 0:  # z e^{-a|x-Rc|^2}
            val = m0[0] * m0[1] * m1[2]
        else:       # z n.(x - Rc) e^{-a|x-Rc|^2}
            val = (n[0] * (m1[0] - Rc[0] * m0[0]) * m0[1] * m1[2] +
                   n[1] * m0[0] * (m1[1] - Rc[1] * m0[1]) * m1[2] +
                   n[2] * m0[0] * m0[1] * (m2z - Rc[2] * m1[2]))
        total += c * val
    total *= (2 * math.pi) ** -1.5
    assert abs(me_oracle - total) < 1e-9 * abs(total)


def test_gerade_orbital_ionises_the_same_along_n_and_minus_n(orc):
    p = saddle(W.n2(0.0))
    n = np.array([0.6, 0.0, 0.8])
    for t0, kp in [(3.0, (0.1, 0.2)), (-30.0, (0.0, -0.2))]:
        a = orc.sfa_step(p, t0, kp, n)
        b = orc.sfa_step(p, t0, kp, -n)
        assert abs(a["m"] - b["m"]) < 1e-12 * abs(a["m"])
        assert a["S"] == b["S"] and a["q0z"] == b["q0z"]


def test_saddle_sampling_weight_and_phase(orc):
    """The sampled ensemble carries the saddle point: p_z = k_z, q0 = (0, 0,
    q0_z), the weight |m| e^{-Im S} over the k_perp density in units of the
    peak-field tunnelling factor, and the birth phase beyond I_p t0 + p0.q0."""
    p = saddle(W.n2(0.0))
    w, E0, tau, N = orc.laser(p)
    Ip = p["target"]["Ip"]
    s = orc.sample(p, 1002, 0, 400)
    kap = math.sqrt(2 * Ip)
    live = np.nonzero(s["w"] > 0)[0]
    assert 50 < len(live) < 400
    for i in live[:40]:
        t0 = orc.time(p, int(s["k0"][i]))
        r = orc.sfa_step(p, t0, s["p0"][i, :2], s["nax"][i])
        assert s["p0"][i, 2] == r["kz"] and s["q0"][i, 2] == r["q0z"]
        kp2 = s["p0"][i, 0] ** 2 + s["p0"][i, 1] ** 2
        lw = math.log(abs(r["m"])) - r["S"].imag + kap ** 3 / (3 * E0) + kp2 / (2 * 0.09)
        assert math.log(s["w"][i]) == pytest.approx(lw, abs=1e-12)
        ph = r["S"].real - Ip * t0 + cmath.phase(r["m"])
        assert abs(cmath.exp(1j * s["dph"][i]) - cmath.exp(1j * ph)) < 1e-12
    dead = s["w"] == 0
    assert np.all(s["dph"][dead] == 0)


def test_weight_compensates_the_transverse_proposal(orc):
    """The weight divides out the Gaussian k_perp proposal (up to its
    normalisation 1/(2 pi sigma^2)), so sigma^2 <w> estimates the same
    integral of |m e^{iS}| for any proposal width wider than the true
    k_perp spread (Monte Carlo, 8,000 trajectories per width drawn from the
    same random numbers: the ratio scatters by ~3%)."""
    vals = []
    for sig in (0.3, 0.45):
        p = W.with_changes(saddle(W.h2_softcore(0.0)), sigma_perp=sig, w_cut=0.0)
        s = orc.sample(p, 77, 0, 8000)
        vals.append(sig * sig * s["w"].mean())
    assert vals[0] == pytest.approx(vals[1], rel=0.08)


def test_birth_phase_of_an_s_orbital_in_the_adiabatic_limit(orc):
    """For one s-type centre (R = 0) in a quasi-static field the ionisation
    element at the saddle point is real and negative on both half-cycles
    (m ~ E(t_s)(-i kappa_z)/(2a) with kappa_z = -/+ i kappa0 sgn E) and the
    square root sqrt(E kappa_z) = sqrt(-i |E| kappa0) has phase -pi/4, while
    Re S - I_p t0 vanishes: every birth phase tends to -3 pi/4."""
    p = saddle(W.h2_softcore(0.0, laser=dict(W.H2_LASER, lambda_nm=16000.0, n_cycles=4.0)))
    p["target"]["R"] = 0.0
    s = orc.sample(p, 4242, 0, 600)
    big = s["w"] > 0.05 * s["w"].max()
    assert big.sum() > 30
    d = np.abs(np.exp(1j * s["dph"][big]) - cmath.exp(-0.75j * math.pi))
    # the O(omega) part of Re S - I_p t0 spreads the phases by up to ~0.2 here
    assert np.all(d < 0.3) and np.median(d) < 0.05


# ------------------------------------------------------------------ SFHK2
def modified(p):
    return W.with_changes(p, ionization="saddle_modified")


def test_modified_saddle_point_solves_its_equation(orc):
    """(k_z + A(t_s) - A(t0))^2 + k_perp^2 + 2 I_p + 2 sgn E(t0) D E(t_s) = 0,
    D = (R/2)|n_z| (the term -eta E(t_s).r0 of Sec. III.C)."""
    rng = np.random.default_rng(8)
    for theta in (0.0, 35.0, 70.0):
        p = modified(W.n2(theta))
        Ip, R = p["target"]["Ip"], p["target"]["R"]
        th = math.radians(theta)
        n = np.array([math.sin(th), 0.0, math.cos(th)])
        for _ in range(8):
            t0 = rng.uniform(-150, 150)
            kp = rng.normal(0, 0.3, 2)
            r = orc.sfa_step(p, t0, kp, n)
            if r is None:
                continue
            E0, A0 = orc.field(p, t0)
            As, Es = orc.field_complex(p, t0, r["tt"])
            kz = r["kz"] + As - A0
            f = kz * kz + kp @ kp + 2 * Ip + 2 * math.copysign(1, E0) * 0.5 * R * abs(n[2]) * Es
            assert abs(f) < 1e-11 and r["tt"] > 0


def test_modified_step_raises_the_effective_ionisation_potential(orc):
    """Quasi-static limit at the field peak: the modified saddle point is the
    unmodified one for I_p' = I_p + |E| D: t_t -> kappa'/|E|, Im S ->
    kappa'^3/(3|E|), kappa'^2 = 2 I_p' + k_perp^2 (corrections O(gamma^2))."""
    for lam, tol in ((8000.0, 0.02), (16000.0, 0.005)):
        p = modified(W.n2(0.0, laser=dict(W.N2_LASER, lambda_nm=lam, n_cycles=8.0)))
        w, E0, tau, N = orc.laser(p)
        Ip, R = p["target"]["Ip"], p["target"]["R"]
        r = orc.sfa_step(p, 0.0, (0.1, 0.0), (0, 0, 1))
        E, _ = orc.field(p, 0.0)
        kap = math.sqrt(2 * (Ip + E * 0.5 * R) + 0.01)
        assert abs(r["kz"]) < 1e-10
        assert r["tt"] == pytest.approx(kap / E, rel=tol)
        assert r["S"].imag == pytest.approx(kap ** 3 / (3 * E), rel=tol)
        r1 = orc.sfa_step(saddle(p), 0.0, (0.1, 0.0), (0, 0, 1))
        assert r["S"].imag > r1["S"].imag  # stronger suppression: a larger effective I_p


def test_modified_step_vanishes_at_90_degrees_and_is_inversion_symmetric(orc):
    p90 = W.n2(90.0)
    n90 = (1.0, 0.0, math.cos(math.radians(90.0)))
    for t0 in (4.0, -33.0):
        a = orc.sfa_step(modified(p90), t0, (0.1, 0.05), n90)
        b = orc.sfa_step(saddle(p90), t0, (0.1, 0.05), n90)
        assert abs(a["S"] - b["S"]) < 1e-10 and abs(a["m"] - b["m"]) < 1e-10 * abs(b["m"])
    p = modified(W.n2(30.0))
    n = np.array([0.5, 0.0, math.sqrt(0.75)])
    for t0 in (4.0, -33.0):
        a = orc.sfa_step(p, t0, (0.1, 0.05), n)
        b = orc.sfa_step(p, t0, (0.1, 0.05), -n)
        assert abs(a["S"] - b["S"]) < 1e-12 and abs(a["m"] - b["m"]) < 1e-12 * abs(a["m"])
        assert a["tt"] == b["tt"] and a["kz"] == b["kz"]

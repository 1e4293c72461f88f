"""ctypes front end of the SFHK oracle (``oracle/sfhk_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product path never imports it.  Problems are
the plain dictionaries of the ``workloads`` module.
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

MAX_GTO = 64
NFINAL = 47
F_Q, F_P, F_M, F_S, F_CRE, F_CIM, F_FLIPS, F_MMAX = 0, 3, 6, 42, 43, 44, 45, 46


class Problem(C.Structure):
    _fields_ = [
        ("lambda_nm", C.c_double), ("intensity_wcm2", C.c_double),
        ("n_cycles", C.c_double), ("cep", C.c_double),
        ("R", C.c_double), ("Ip", C.c_double),
        ("Zinf", C.c_double * 2), ("dZ", C.c_double * 2),
        ("alpha", C.c_double * 2), ("eps2", C.c_double * 2),
        ("n_gto", C.c_int32),
        ("gto_center", C.c_int32 * MAX_GTO), ("gto_l", C.c_int32 * MAX_GTO),
        ("gto_a", C.c_double * MAX_GTO), ("gto_c", C.c_double * MAX_GTO),
        ("align_kind", C.c_int32), ("align_m", C.c_int32),
        ("theta", C.c_double), ("phi", C.c_double),
        ("dt", C.c_double), ("gamma", C.c_double), ("w_cut", C.c_double),
        ("sigma_perp", C.c_double),
        ("n_steps", C.c_int32),
        ("c_max", C.c_double),
        ("ionization", C.c_int32),
    ]

IONIZATION = {"first_order": 0, "saddle": 1, "saddle_modified": 2}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        P = C.POINTER(Problem)
        L.orc_laser.argtypes = [P, dp, dp, dp, C.POINTER(C.c_int32)]
        L.orc_time.argtypes = [P, C.c_int32]
        L.orc_time.restype = C.c_double
        L.orc_field.argtypes = [P, C.c_double, dp, dp]
        L.orc_potential.argtypes = [P, dp, dp, dp, dp, dp]
        L.orc_recombination.argtypes = [P, dp, dp, dp, dp, dp]
        L.orc_prefactor_det.argtypes = [dp, C.c_double, dp, dp]
        u32p = C.POINTER(C.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_sample.argtypes = [P, C.c_uint64, C.c_uint64, C.c_uint64,
                                 C.POINTER(C.c_int32), dp, dp, dp, dp, dp]
        L.orc_trajectory.argtypes = [P, C.c_int32, C.c_int32, dp, dp, dp, C.c_double,
                                     C.c_double, dp, dp, dp, dp, dp]
        L.orc_sfa_step.argtypes = [P, C.c_double, dp, dp, dp]
        L.orc_sfa_step.restype = C.c_int
        L.orc_field_complex.argtypes = [P, C.c_double, C.c_double, dp, dp, dp, dp]
        L.orc_trajectory.restype = C.c_int
        L.orc_run.argtypes = [P, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int32, dp,
                              C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.orc_run.restype = C.c_int
        L.orc_run_ensemble.argtypes = [P, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int32,
                                       C.c_double, dp, dp, dp, C.POINTER(C.c_uint64),
                                       C.POINTER(C.c_uint64)]
        L.orc_run_ensemble.restype = C.c_int
        L.orc_spectrum.argtypes = [dp, C.c_int32, C.c_double, C.c_double, C.c_double,
                                   dp, C.c_int32, dp, dp, dp]
        L.orc_return_step.argtypes = [P, C.c_int32, dp, dp, dp, C.c_double,
                                      C.POINTER(C.c_int32), dp]
        L.orc_gabor.argtypes = [dp, C.c_int32, C.c_double, C.c_double, C.c_double, dp,
                                C.c_int32, dp, C.c_int32, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


def make_problem(d):
    """ctypes Problem from a workloads problem dictionary."""
    P = Problem()
    las, tgt, al = d["laser"], d["target"], d["align"]
    P.lambda_nm = las["lambda_nm"]
    P.intensity_wcm2 = las["intensity_wcm2"]
    P.n_cycles = las["n_cycles"]
    P.cep = las["cep"]
    P.R = tgt["R"]
    P.Ip = tgt["Ip"]
    for i, c in enumerate(tgt["centers"]):
        P.Zinf[i] = c["Zinf"]
        P.dZ[i] = c["dZ"]
        P.alpha[i] = c["alpha"]
        P.eps2[i] = c["eps2"]
    gto = tgt["gto"]
    assert len(gto) <= MAX_GTO
    P.n_gto = len(gto)
    for j, (ctr, l, a, c) in enumerate(gto):
        P.gto_center[j] = int(ctr)
        P.gto_l[j] = int(l)
        P.gto_a[j] = a
        P.gto_c[j] = c
    P.align_kind = 0 if al["kind"] == "fixed" else 1
    P.align_m = int(al.get("m", 0))
    P.theta = al.get("theta", 0.0)
    P.phi = al.get("phi", 0.0)
    P.dt = d["dt"]
    P.gamma = d["gamma"]
    P.w_cut = d["w_cut"]
    P.sigma_perp = d["sigma_perp"]
    P.n_steps = int(d.get("n_steps", 0))
    P.c_max = float(d.get("c_max", 0.0))
    P.ionization = IONIZATION[d.get("ionization", "first_order")]
    return P


def laser(d):
    """(omega, E0, tau, N)."""
    P = make_problem(d)
    w, e, t, n = C.c_double(), C.c_double(), C.c_double(), C.c_int32()
    lib().orc_laser(C.byref(P), C.byref(w), C.byref(e), C.byref(t), C.byref(n))
    return w.value, e.value, t.value, n.value


def n_steps(d):
    return laser(d)[3]


def time(d, k):
    return lib().orc_time(C.byref(make_problem(d)), int(k))


def times(d):
    N = n_steps(d)
    P = make_problem(d)
    return np.array([lib().orc_time(C.byref(P), k) for k in range(N + 1)])


def field(d, t):
    """(E(t), A(t)) for a scalar or array t."""
    P = make_problem(d)
    ts = np.atleast_1d(np.asarray(t, dtype=np.float64))
    E = np.empty_like(ts)
    A = np.empty_like(ts)
    e, a = C.c_double(), C.c_double()
    for i, ti in enumerate(ts):
        lib().orc_field(C.byref(P), float(ti), C.byref(e), C.byref(a))
        E[i], A[i] = e.value, a.value
    if np.ndim(t) == 0:
        return E[0], A[0]
    return E, A


def potential(d, nax, q):
    P = make_problem(d)
    n = _arr(nax, 3)
    qq = _arr(q, 3)
    V = C.c_double()
    g = np.zeros(3)
    H = np.zeros(9)
    lib().orc_potential(C.byref(P), _dp(n), _dp(qq), C.byref(V), _dp(g), _dp(H))
    return V.value, g, H.reshape(3, 3)


def recombination(d, nax, p, q):
    P = make_problem(d)
    n, pp, qq = _arr(nax, 3), _arr(p, 3), _arr(q, 3)
    re, im = C.c_double(), C.c_double()
    lib().orc_recombination(C.byref(P), _dp(n), _dp(pp), _dp(qq), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def prefactor_det(M, gamma):
    m = _arr(M, 36)
    re, im = C.c_double(), C.c_double()
    lib().orc_prefactor_det(_dp(m), float(gamma), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def sample(d, seed, first, n):
    """dict of k0 [n], q0 [n,3], p0 [n,3], nax [n,3], w [n], dph [n] for
    trajectories first..first+n-1."""
    P = make_problem(d)
    k0 = np.zeros(n, dtype=np.int32)
    q0 = np.zeros((n, 3))
    p0 = np.zeros((n, 3))
    nax = np.zeros((n, 3))
    w = np.zeros(n)
    dph = np.zeros(n)
    lib().orc_sample(C.byref(P), int(seed), int(first), int(n),
                     k0.ctypes.data_as(C.POINTER(C.c_int32)), _dp(q0), _dp(p0), _dp(nax), _dp(w),
                     _dp(dph))
    return {"k0": k0, "q0": q0, "p0": p0, "nax": nax, "w": w, "dph": dph}


def sfa_step(d, t0, kperp, nax):
    """Exact SFA ionisation step: dict(tt, kz, q0z, S (complex), m (complex)) or None."""
    P = make_problem(d)
    out = np.zeros(7)
    kp, n = _arr(kperp, 2), _arr(nax, 3)
    if lib().orc_sfa_step(C.byref(P), float(t0), _dp(kp), _dp(n), _dp(out)) != 0:
        return None
    return {"tt": out[0], "kz": out[1], "q0z": out[2], "S": complex(out[3], out[4]),
            "m": complex(out[5], out[6])}


def field_complex(d, tr, ti):
    """(A, E) of the laser at complex time tr + i ti."""
    P = make_problem(d)
    v = [C.c_double() for _ in range(4)]
    lib().orc_field_complex(C.byref(P), float(tr), float(ti), *[C.byref(x) for x in v])
    return complex(v[0].value, v[1].value), complex(v[2].value, v[3].value)


def trajectory(d, k0, q0, p0, nax, w=1.0, k_end=None, amplitudes=True, prefactors=False,
               dph=0.0):
    """Propagate one trajectory; returns (a [N+1] complex or None, final [NFINAL]),
    plus C [N+1] complex when prefactors=True."""
    P = make_problem(d)
    N = n_steps(d)
    if k_end is None:
        k_end = N
    fin = np.zeros(NFINAL)
    q, p, n = _arr(q0, 3), _arr(p0, 3), _arr(nax, 3)
    are = np.zeros(N + 1) if amplitudes else None
    aim = np.zeros(N + 1) if amplitudes else None
    cre = np.zeros(N + 1) if prefactors else None
    cim = np.zeros(N + 1) if prefactors else None
    ptr = lambda a: _dp(a) if a is not None else None
    rc = lib().orc_trajectory(C.byref(P), int(k0), int(k_end), _dp(q), _dp(p), _dp(n), float(w),
                              float(dph), ptr(are), ptr(aim), ptr(cre), ptr(cim), _dp(fin))
    if rc != 0:
        raise ValueError("orc_trajectory rejected its arguments")
    a = (are + 1j * aim) if amplitudes else None
    if prefactors:
        return a, fin, cre + 1j * cim
    return a, fin


def run(d, seed, first, n, nthreads=None):
    """(accum [N+1], live_steps, n_live): accum[k] = sum_j Re a_jk."""
    P = make_problem(d)
    N = n_steps(d)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    acc = np.zeros(N + 1)
    ls, nl = C.c_uint64(), C.c_uint64()
    rc = lib().orc_run(C.byref(P), int(seed), int(first), int(n), int(nthreads), _dp(acc),
                       C.byref(ls), C.byref(nl))
    if rc != 0:
        raise RuntimeError("orc_run failed")
    return acc, ls.value, nl.value


def run_ensemble(d, seed, first, n, m_regular=1e4, nthreads=None, finals=True):
    """orc_run split by each trajectory's largest monodromy entry: dict of
    accum_all, accum_regular (trajectories with max_k max_ij |M_ij| <= m_regular),
    finals [n, NFINAL] (zeros for trajectories not propagated; None if
    finals=False), live_steps, n_live."""
    P = make_problem(d)
    N = n_steps(d)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    acc_all = np.zeros(N + 1)
    acc_reg = np.zeros(N + 1)
    fin = np.zeros((n, NFINAL)) if finals else None
    ls, nl = C.c_uint64(), C.c_uint64()
    rc = lib().orc_run_ensemble(C.byref(P), int(seed), int(first), int(n), int(nthreads),
                                float(m_regular), _dp(acc_all), _dp(acc_reg),
                                _dp(fin) if fin is not None else None, C.byref(ls), C.byref(nl))
    if rc != 0:
        raise RuntimeError("orc_run_ensemble failed")
    return {"accum_all": acc_all, "accum_regular": acc_reg, "finals": fin,
            "live_steps": ls.value, "n_live": nl.value}


def dipole(d, seed, first, n, nthreads=None):
    """v_k = (2/N_s) sum_j Re a_jk for N_s = n sampled trajectories."""
    acc, ls, nl = run(d, seed, first, n, nthreads)
    return (2.0 / n) * acc if n > 0 else acc, ls, nl


def spectrum(v, t_first, dt, tau_H, omega):
    v = _arr(v)
    om = _arr(omega)
    Vr = np.zeros(om.size)
    Vi = np.zeros(om.size)
    Y = np.zeros(om.size)
    lib().orc_spectrum(_dp(v), v.size, float(t_first), float(dt), float(tau_H), _dp(om),
                       om.size, _dp(Vr), _dp(Vi), _dp(Y))
    return Vr + 1j * Vi, Y


def fft_log2_len(n_t):
    """log2 of the zero-padded transform length: the power of two >= 8 n_t."""
    return int(math.ceil(math.log2(8 * max(int(n_t), 1))))


def spectrum_fft(v, t_first, dt, tau_H, log2_len=None):
    """Eq. 3 on the grid of a zero-padded transform: x_k = v_k W_H(t_k)
    (k < n_t; 0 up to L = 2^log2_len), w_j = 2 pi j / (L dt) for
    j = 0 .. L/2, V_j = dt sum_k x_k exp(i w_j t_k) with t_k = t_first + k dt;
    the dipole acceleration's spectrum A = -i w V (Sec. II.A: the forms
    differ by that factor), yield |A|^2 = w^2 |V|^2 and phase arg A.  numpy's
    FFT is the transform step.  Returns (omega, V, yield, phase)."""
    v = _arr(v)
    n = v.size
    L = 1 << (fft_log2_len(n) if log2_len is None else int(log2_len))
    t = t_first + np.arange(n) * dt
    wh = np.where(np.abs(t) <= tau_H, 0.5 * (1.0 + np.cos(np.pi * t / tau_H)), 0.0)
    x = np.zeros(L)
    x[:n] = v * wh
    X = np.fft.ifft(x) * L                      # sum_k x_k exp(+2 pi i j k / L)
    j = np.arange(L // 2 + 1)
    w = 2.0 * np.pi * j / (L * dt)
    V = dt * np.exp(1j * w * t_first) * X[:L // 2 + 1]
    A = -1j * w * V
    return w, V, np.abs(A) ** 2, np.angle(A)


def acceleration_fft(v, t_first, dt, tau_H, log2_len=None):
    """The dipole acceleration on the step grid: the time derivative of the
    windowed dipole W_H v through its zero-padded spectrum (A = -i w V,
    Sec. II.A), a_k = (1/L) sum_j (-i w_j) X_j exp(-2 pi i j k / L) with the
    two-sided frequencies w_j = 2 pi j / (L dt) (j < L/2), 2 pi (j - L) / (L dt)
    (j > L/2) and the Nyquist term dropped; k < n_t.  numpy's FFT is the
    transform step."""
    v = _arr(v)
    n = v.size
    L = 1 << (fft_log2_len(n) if log2_len is None else int(log2_len))
    t = t_first + np.arange(n) * dt
    wh = np.where(np.abs(t) <= tau_H, 0.5 * (1.0 + np.cos(np.pi * t / tau_H)), 0.0)
    x = np.zeros(L)
    x[:n] = v * wh
    X = np.fft.ifft(x) * L
    w = 2.0 * np.pi * np.fft.fftfreq(L, d=dt)
    w[L // 2] = 0.0
    return (np.fft.fft(-1j * w * X) / L).real[:n]


def gabor(v, t_first, dt, sigma, t_c, omega):
    """(G [n_c, n_omega] complex, yield) of the Gaussian-window transform."""
    v, tc, om = _arr(v), _arr(t_c), _arr(omega)
    Gr = np.zeros((tc.size, om.size))
    Gi = np.zeros_like(Gr)
    Y = np.zeros_like(Gr)
    lib().orc_gabor(_dp(v), v.size, float(t_first), float(dt), float(sigma), _dp(tc), tc.size,
                    _dp(om), om.size, _dp(Gr), _dp(Gi), _dp(Y))
    return Gr + 1j * Gi, Y


def return_step(d, k0, q0, p0, nax, r_ret):
    """(k_ret or -1, return kinetic energy) of one trajectory."""
    P = make_problem(d)
    k, e = C.c_int32(), C.c_double()
    lib().orc_return_step(C.byref(P), int(k0), _dp(_arr(q0, 3)), _dp(_arr(p0, 3)),
                          _dp(_arr(nax, 3)), float(r_ret), C.byref(k), C.byref(e))
    return k.value, e.value

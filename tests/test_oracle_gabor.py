"""Pins of the oracle's Gabor transform (time-frequency analysis of the
dipole, Sec. III.C): the closed form for a pure tone, covariance under a
time shift, and the time integral that returns the Fourier transform."""
import math

import numpy as np
import pytest


def test_gabor_of_a_pure_tone(orc):
    """int cos(w0 t + phi) e^{-(t - tc)^2/(2 s^2)} e^{i W t} dt =
    s sqrt(2 pi)/2 [e^{i phi} e^{i(W + w0) tc} e^{-s^2 (W + w0)^2/2} +
                    e^{-i phi} e^{i(W - w0) tc} e^{-s^2 (W - w0)^2/2}];
    the grid sum matches it to rounding once the window is resolved."""
    dt, w0, phi, s = 0.05, 0.35, 0.4, 1.0 / (3 * 0.057)
    t = -400.0 + dt * np.arange(16001)
    v = np.cos(w0 * t + phi)
    tc = np.array([-120.0, 0.0, 33.3, 150.0])
    W = np.linspace(0.0, 1.2, 25)
    G, Y = orc.gabor(v, t[0], dt, s, tc, W)
    ref = np.empty_like(G)
    for a, c in enumerate(tc):
        ref[a] = 0.5 * s * math.sqrt(2 * math.pi) * (
            np.exp(1j * phi) * np.exp(1j * (W + w0) * c) * np.exp(-0.5 * s * s * (W + w0) ** 2) +
            np.exp(-1j * phi) * np.exp(1j * (W - w0) * c) * np.exp(-0.5 * s * s * (W - w0) ** 2))
    assert np.max(np.abs(G - ref)) < 1e-11 * np.max(np.abs(ref))
    assert np.allclose(Y, W[None, :] ** 2 * np.abs(G) ** 2, rtol=1e-14, atol=0)


def test_gabor_time_shift_covariance(orc):
    """Delaying the signal by m grid steps delays the map: G'(tc + m dt, W) =
    e^{i W m dt} G(tc, W)."""
    rng = np.random.default_rng(3)
    dt, s, m = 0.1, 6.0, 37
    v = np.zeros(3000)
    v[1000:2000] = rng.normal(size=1000)
    vs = np.roll(v, m)
    tc = np.array([-20.0, 10.0, 55.5])
    W = np.array([0.1, 0.7, 1.9])
    t0 = -150.0
    G, _ = orc.gabor(v, t0, dt, s, tc, W)
    Gs, _ = orc.gabor(vs, t0, dt, s, tc + m * dt, W)
    assert np.max(np.abs(Gs - np.exp(1j * W * m * dt)[None, :] * G)) < 1e-12 * np.max(np.abs(G))


def test_gabor_integrated_over_time_is_the_fourier_transform(orc):
    """sum_c G(t_c, W) dt_c over centres covering the signal with margin =
    s sqrt(2 pi) dt sum_k v_k e^{i W t_k} (the unwindowed transform)."""
    rng = np.random.default_rng(4)
    dt, s = 0.1, 3.0
    t0 = -50.0
    v = np.zeros(1000)
    v[300:700] = rng.normal(size=400)
    tc = t0 + dt * np.arange(-400, 1400)  # every grid point, 40 a.u. beyond both ends
    W = np.array([0.0, 0.3, 1.1])
    G, _ = orc.gabor(v, t0, dt, s, tc, W)
    lhs = G.sum(axis=0) * dt
    tk = t0 + dt * np.arange(v.size)
    ft = dt * (v[:, None] * np.exp(1j * W[None, :] * tk[:, None])).sum(axis=0)
    assert np.max(np.abs(lhs - s * math.sqrt(2 * math.pi) * ft)) < 1e-10 * np.max(np.abs(ft))

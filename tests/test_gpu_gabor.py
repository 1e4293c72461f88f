"""The Gabor transform on the GPU (sfhk_gabor) against the oracle's plain
sum: a computed dipole at the default window width, a window wider than one
LDS chunk, and a pure tone against its closed form."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13686_amd as sf
    return sf


def rel(a, b):
    r = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(f"relative L2 {r:.3e}", flush=True)
    return r


def test_gabor_of_a_dipole_matches_oracle(sf, orc):
    import torch
    p = W.h2_softcore()
    out = sf.run([p], [2048], [1001], h_max=40.0)
    torch.cuda.synchronize()
    v = out["v"][0]
    N, t0, tau = sf.problem_steps(p)
    sig = sf.gabor_width(p)
    tc = np.linspace(-150.0, 150.0, 121)
    om = np.linspace(0.0, 40.0, 161) * 45.56335252912 / p["laser"]["lambda_nm"]
    G, Y = sf.gabor(v, t0, p["dt"], sig, tc, om)
    torch.cuda.synchronize()
    Go, Yo = orc.gabor(v.cpu().numpy(), t0, p["dt"], sig, tc, om)
    assert rel(G.cpu().numpy(), Go) < 1e-12
    assert rel(Y.cpu().numpy(), Yo) < 1e-11


def test_gabor_window_wider_than_a_chunk(sf, orc):
    import torch
    rng = np.random.default_rng(9)
    n_t, dt, sig = 30000, 0.05, 40.0  # 8 sigma / dt = 6400 steps each side: several chunks
    v = torch.tensor(rng.normal(size=n_t), dtype=torch.float64, device="cuda")
    tc = np.array([-700.0, -300.0, 0.0, 450.0])
    om = np.array([0.0, 0.05, 0.4, 2.0, 7.5])
    G, _ = sf.gabor(v, -750.0, dt, sig, tc, om)
    torch.cuda.synchronize()
    Go, _ = orc.gabor(v.cpu().numpy(), -750.0, dt, sig, tc, om)
    assert rel(G.cpu().numpy(), Go) < 1e-12


def test_gabor_of_a_pure_tone(sf):
    import torch
    dt, w0, s = 0.05, 0.35, 8.0
    t = -400.0 + dt * np.arange(16001)
    v = torch.tensor(np.cos(w0 * t), dtype=torch.float64, device="cuda")
    tc = np.array([-100.0, 20.0])
    W_ = np.linspace(0.0, 1.0, 11)
    G, _ = sf.gabor(v, t[0], dt, s, tc, W_)
    torch.cuda.synchronize()
    ref = np.array([0.5 * s * math.sqrt(2 * math.pi) * (
        np.exp(1j * (W_ + w0) * c - 0.5 * s * s * (W_ + w0) ** 2) +
        np.exp(1j * (W_ - w0) * c - 0.5 * s * s * (W_ - w0) ** 2)) for c in tc])
    assert np.max(np.abs(G.cpu().numpy() - ref)) < 1e-11 * np.max(np.abs(ref))

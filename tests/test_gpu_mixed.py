"""Mixed-precision form (FP32 position/momentum/monodromy stepping; FP64
action, prefactor, recombination, amplitude and dipole) against the FP64
kernel and the oracle.  The error is measured and stated, not hidden: the
asserted bounds are the stated accuracy of the mixed form."""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)
# stated accuracy of the mixed form on these workloads, a few times the
# measured relative L2 errors (H2 2.4e-5; N2 4.6e-2 at 0 degrees, 5.3e-5 at
# 90 degrees); the spectra move by a median 0.007 dB (N2) or less.
MIXED_REL_L2 = {"H2": 1e-4, "N2": 1e-1}
MIXED_SPECTRAL_DB_MEDIAN = 0.05


@pytest.fixture(scope="module")
def sf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13686_amd as sf
    return sf


def both_precisions(sf, probs, n, seeds):
    import torch
    ens, ws = sf.sample_initial(probs, n, seeds)
    out = {}
    for prec in ("fp64", "mixed"):
        acc, fs = sf.propagate(probs, ens, precision=prec, final_state=True, workspace=ws)
        v = sf.dipole(probs, acc, n)
        torch.cuda.synchronize()
        out[prec] = (v.cpu().numpy(), fs.cpu().numpy())
    return ens, out


def spectral_db(sf, prob, v64, vmx, h_lo, h_hi):
    import torch
    N, t0, tau = sf.problem_steps(prob)
    om = sf.harmonic_grid(prob, h_hi).cuda()
    _, y64 = sf.spectrum(torch.tensor(v64, device="cuda"), t0, prob["dt"], tau / 2, om)
    _, ymx = sf.spectrum(torch.tensor(vmx, device="cuda"), t0, prob["dt"], tau / 2, om)
    h = (om / om[1] * 0.05).cpu().numpy()
    sel = (h >= h_lo) & (h <= h_hi)
    db = np.abs(10 * np.log10(ymx.cpu().numpy()[sel] / y64.cpu().numpy()[sel]))
    return float(np.median(db)), float(np.percentile(db, 90))


@pytest.mark.parametrize("mol", ["H2", "N2"])
def test_mixed_dipole_error_vs_fp64(sf, mol):
    if mol == "H2":
        probs, n, seeds, h_lo, h_hi = [workloads.h2_softcore()], [4096], [1001], 10.0, 40.0
    else:
        probs, n, seeds, h_lo, h_hi = [workloads.n2(0.0), workloads.n2(90.0)], [8192, 8192], [1002, 1002], 15.0, 80.0
    ens, out = both_precisions(sf, probs, n, seeds)
    offs, lens = sf.accum_layout(probs)
    for p, o, l in zip(probs, offs, lens):
        v64 = out["fp64"][0][o:o + l]
        vmx = out["mixed"][0][o:o + l]
        rel = np.linalg.norm(vmx - v64) / np.linalg.norm(v64)
        med, p90 = spectral_db(sf, p, v64, vmx, h_lo, h_hi)
        print(f"{p['name']} theta={p['align']['theta']:.3f}: mixed vs FP64 relative L2 {rel:.3e}, "
              f"spectral |dB| median {med:.3f}, 90th pct {p90:.3f} (H{h_lo:g}-H{h_hi:g})")
        assert rel < MIXED_REL_L2[mol]
        assert med < MIXED_SPECTRAL_DB_MEDIAN


def test_mixed_regular_trajectories_vs_oracle(sf, orc):
    """Trajectories with a modest monodromy norm follow the oracle to FP32
    accuracy amplified by |M|."""
    probs = [workloads.n2(30.0)]
    ens, out = both_precisions(sf, probs, [400], [5])
    g = {f: getattr(ens, f).cpu().numpy() for f in ens.FIELDS_I32 + ens.FIELDS_F64}
    fs = out["mixed"][1]
    live = np.nonzero(g["w"] > 0)[0]
    checked = 0
    worst = 0.0
    for i in live[:40]:
        _, fo = orc.trajectory(probs[0], int(g["k0"][i]), (g["qx"][i], g["qy"][i], g["qz"][i]),
                               (g["px"][i], g["py"][i], g["pz"][i]),
                               (g["nx"][i], g["ny"][i], g["nz"][i]), g["w"][i], amplitudes=False)
        amp = 1.0 + np.linalg.norm(fo[6:42].reshape(6, 6), 2)
        if amp > 1e3:
            continue
        err = np.max(np.abs(fs[0:6, i] - fo[0:6]) / np.maximum(1.0, np.abs(fo[0:6])))
        worst = max(worst, err / amp)
        assert err < 1e-4 * amp, (i, err, amp)
        checked += 1
    print(f"mixed: {checked} regular trajectories, worst error/|M| {worst:.3e}")
    assert checked >= 5


def test_mixed_hands_chaotic_trajectories_to_fp64(sf):
    """Trajectories whose monodromy matrix grows past the FP32 bound are
    finished by the FP64 kernel: their final state equals the FP64 run's bit
    for bit, and the other trajectories keep FP32 accuracy."""
    probs = [workloads.n2(0.0)]
    # at most 128 packs: the FP64 run takes the latency form, as the re-run does
    ens, out = both_precisions(sf, probs, [8000], [1002])
    w = ens.w.cpu().numpy()
    f64, fmx = out["fp64"][1], out["mixed"][1]
    live = np.nonzero(w > 0)[0]
    mmax = np.max(np.abs(f64[6:42, live]), axis=0)
    chaotic = live[mmax > 1e5]
    regular = live[mmax < 1e3]
    print(f"{chaotic.size} chaotic (|M| > 1e5), {regular.size} regular (|M| < 1e3) of {live.size}")
    assert chaotic.size > 0 and regular.size > 0
    # every record field but the count of recombination steps, which the
    # re-run counts from its first deposit
    assert np.array_equal(fmx[:47, chaotic], f64[:47, chaotic])
    rel = np.max(np.abs(fmx[0:6, regular] - f64[0:6, regular]) / np.maximum(1, np.abs(f64[0:6, regular])))
    print(f"regular trajectories: max relative (q, p) difference {rel:.3e}")
    assert rel < 1e-3


def test_mixed_error_with_prefactor_cap(sf):
    """With a prefactor cap (|C| <= 1e3) the mixed run hands every trajectory
    nearing the cap (|C| > c_max/4) to FP64, so the cap stops it at the FP64
    run's step; free spreading alone passes c_max/4 after ~80 a.u., so most
    of each dipole is FP64 on both sides.  The capped results agree to 1e-3
    (a cap decided in FP32 differed by up to 1e-1)."""
    probs = [dict(workloads.n2(0.0), c_max=1e3), dict(workloads.n2(90.0), c_max=1e3),
             dict(workloads.h2_softcore(), c_max=1e3)]
    n, seeds = [65536, 65536, 65536], [1002, 1002, 1001]
    ens, out = both_precisions(sf, probs, n, seeds)
    offs, lens = sf.accum_layout(probs)
    for p, o, l in zip(probs, offs, lens):
        v64 = out["fp64"][0][o:o + l]
        vmx = out["mixed"][0][o:o + l]
        rel = np.linalg.norm(vmx - v64) / np.linalg.norm(v64)
        print(f"capped {p['name']} theta={p['align']['theta']:.3f}: mixed vs FP64 relative L2 {rel:.3e}")
        assert rel < 1e-3


def test_mixed_error_with_chaos_cap(sf):
    """Chaotic trajectories cut by a prefactor cap five times the free-spreading
    |C| = |1 - i gamma tau/2|^{3/2} of a whole-pulse trajectory: regular
    trajectories stay below the hand-over threshold c_max/4 and run in FP32
    throughout, so the dipole error is the FP32 stepping error: measured
    1.7e-4 (H2) to 8.9e-4 (N2, 0 deg) here and up to 3.5e-3 on the batched
    problems at the highest intensity; asserted below 5e-3."""
    def cap(p):
        _, _, tau = sf.problem_steps(p)
        return 5.0 * abs(1.0 - 0.5j * p["gamma"] * tau) ** 1.5
    base = [workloads.n2(0.0), workloads.n2(90.0), workloads.h2_softcore()]
    probs = [dict(p, c_max=cap(p)) for p in base]
    n, seeds = [65536, 65536, 65536], [1002, 1002, 1001]
    ens, out = both_precisions(sf, probs, n, seeds)
    offs, lens = sf.accum_layout(probs)
    for p, o, l in zip(probs, offs, lens):
        v64 = out["fp64"][0][o:o + l]
        vmx = out["mixed"][0][o:o + l]
        rel = np.linalg.norm(vmx - v64) / np.linalg.norm(v64)
        print(f"cap {p['c_max']:.0f} {p['name']} theta={p['align']['theta']:.3f}: "
              f"mixed vs FP64 relative L2 {rel:.3e}", flush=True)
        assert 0 < rel < 5e-3


def test_cap_handover_is_the_fp64_trajectory(sf):
    """With a prefactor cap, a trajectory whose prefactor nears the cap is
    finished by the FP64 kernel from its birth, so its final state (q, p, M,
    S, C, sign flips) equals the FP64 run's (in the same kernel form) bit for bit: checked for every
    live trajectory whose FP64 |C| ends above 0.3 c_max (the hand-over
    threshold is 0.25 c_max)."""
    probs = [dict(workloads.n2(0.0), c_max=1e3), dict(workloads.h2_softcore(), c_max=1e3)]
    # at most 128 packs: the FP64 run takes the latency form, as the re-run does
    n, seeds = [5000, 3000], [1002, 1001]
    ens, out = both_precisions(sf, probs, n, seeds)
    fs64, fsm = out["fp64"][1], out["mixed"][1]
    live = np.nonzero(ens.w.cpu().numpy() > 0)[0]
    c64 = np.hypot(fs64[43, live], fs64[44, live])
    near = live[c64 > 0.3 * 1e3]
    print(f"{near.size} of {live.size} live trajectories end with |C| > 300", flush=True)
    assert near.size > 0.3 * live.size
    assert np.array_equal(fsm[:47, near], fs64[:47, near])  # all but the recombination-step count

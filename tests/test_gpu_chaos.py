"""Parity on the measured N2 workload, strongly amplifying trajectories
included (the reading of the parity tolerance under chaos).

The first 65,536 trajectories of each angle of the headline workload (N2,
Eq. 7 with Table I, 0 and 90 degrees, seed 1002; trajectory j draws the same
numbers at any ensemble size) are propagated by the FP64 kernel in the launch
form of ``sfhk_propagate`` and by the oracle.  A trajectory is regular when the
largest entry of its monodromy matrix along the pulse stays <= 1e4 (oracle's
running maximum); the others pass near a nucleus and amplify rounding by up
to ~1e20, so two correct FP64 evaluations of them differ by ~1e-16 |M|.

* the regular set's dipole sum: relative L2 <= 1e-10 against the oracle's sum
  over the same set (the GPU run zeroes the other slots' weights);
* every live trajectory's final record against the oracle's, with a bound
  1e-12 (1 + max|M|) sqrt(steps) (c 1e-16 max|M| sqrt(n) with c = 1e4);
* the running maximum itself: the kernel's and the oracle's agree on the
  classification and, for regular trajectories, to 1e-9;
* the ensemble error with and without the amplifying trajectories, and their
  share of the dipole norm, printed for the record.
"""
import math
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

N_PREFIX = 65536
M_REGULAR = 1e4
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def sf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13686_amd as sf
    return sf


@pytest.fixture(scope="module")
def prefix_runs(sf, orc):
    """GPU and oracle runs of the 65,536-trajectory prefix of both angles."""
    import torch
    probs = [workloads.n2(0.0), workloads.n2(90.0)]
    n, seeds = [N_PREFIX, N_PREFIX], [1002, 1002]
    print(f"chaos parity: N2 0/90 deg, prefix {N_PREFIX} per angle, seed 1002", flush=True)
    ens, ws = sf.sample_initial(probs, n, seeds)
    acc_all, fs = sf.propagate(probs, ens, final_state=True, workspace=ws)
    torch.cuda.synchronize()
    fs_h = fs.cpu().numpy()
    w_h = ens.w.cpu().numpy()
    orc_runs = []
    for p, sd in zip(probs, seeds):
        orc_runs.append(orc.run_ensemble(p, sd, 0, N_PREFIX, m_regular=M_REGULAR,
                                         nthreads=NTHREADS))
    # the regular set on the GPU: zero the weights of the amplifying slots
    chaotic = np.concatenate([r["finals"][:, orc.F_MMAX] > M_REGULAR for r in orc_runs])
    w_reg = ens.w.clone()
    w_reg[torch.from_numpy(np.nonzero(chaotic)[0]).to(w_reg.device)] = 0.0
    ens.w.copy_(w_reg)
    acc_reg, _ = sf.propagate(probs, ens, workspace=ws)
    torch.cuda.synchronize()
    return {"probs": probs, "acc_all": acc_all.cpu().numpy(), "acc_reg": acc_reg.cpu().numpy(),
            "fs": fs_h, "w": w_h, "orc": orc_runs, "offs": sf.accum_layout(probs)}


def test_regular_set_dipole_matches_oracle(prefix_runs):
    r = prefix_runs
    offs, lens = r["offs"]
    for P, (o, l) in enumerate(zip(offs, lens)):
        ro = r["orc"][P]
        g_reg, o_reg = r["acc_reg"][o:o + l], ro["accum_regular"]
        g_all, o_all = r["acc_all"][o:o + l], ro["accum_all"]
        err_reg = np.linalg.norm(g_reg - o_reg) / np.linalg.norm(o_reg)
        err_all = np.linalg.norm(g_all - o_all) / np.linalg.norm(o_all)
        share = np.linalg.norm(o_all - o_reg) / np.linalg.norm(o_all)
        n_cha = int(np.sum(ro["finals"][:, 46] > M_REGULAR))
        print(f"angle {P}: {ro['n_live']} live, {n_cha} with max|M| > 1e4; rel L2 regular "
              f"{err_reg:.3e}, all {err_all:.3e}; share of |v| from max|M| > 1e4: {share:.3e}",
              flush=True)
        assert np.all(np.isfinite(g_all)) and np.all(np.isfinite(g_reg))
        assert 0 < n_cha < 0.02 * ro["n_live"]
        assert err_reg <= 1e-10


def test_running_maximum_matches_oracle(prefix_runs, orc):
    r = prefix_runs
    for P in range(2):
        fo = r["orc"][P]["finals"]
        fg = r["fs"][:, P * N_PREFIX:(P + 1) * N_PREFIX]
        live = r["w"][P * N_PREFIX:(P + 1) * N_PREFIX] > 0
        mo, mg = fo[live, orc.F_MMAX], fg[46, live]
        near = np.abs(np.log(mo / M_REGULAR)) < 1e-6
        assert np.array_equal((mo > M_REGULAR)[~near], (mg > M_REGULAR)[~near])
        reg = mo <= M_REGULAR
        err = np.max(np.abs(mg[reg] - mo[reg]) / mo[reg])
        print(f"angle {P}: running max |M| of {reg.sum()} regular trajectories, max rel err "
              f"{err:.2e}; largest max|M| {mo.max():.3e}", flush=True)
        assert err < 1e-9


def test_every_final_record_within_amplified_rounding(prefix_runs, orc):
    """q, p, S, C relative to max(1, |x|) and M relative to 1 + max|M|, each
    within 1e-12 (1 + max|M|) sqrt(steps); the branch-flip count exactly for
    regular trajectories."""
    r = prefix_runs
    N = orc.n_steps(r["probs"][0])
    for P in range(2):
        fo = r["orc"][P]["finals"]
        fg = r["fs"][:, P * N_PREFIX:(P + 1) * N_PREFIX].T
        live = np.nonzero(r["w"][P * N_PREFIX:(P + 1) * N_PREFIX] > 0)[0]
        k0 = orc.sample(r["probs"][P], 1002, 0, N_PREFIX)["k0"][live]
        a, b = fg[live], fo[live]
        amp = 1.0 + b[:, 46]
        tol = 1e-12 * amp * np.sqrt(N - k0 + 1.0)
        e_qp = np.max(np.abs(a[:, 0:6] - b[:, 0:6]) / np.maximum(1.0, np.abs(b[:, 0:6])), axis=1)
        e_m = np.max(np.abs(a[:, 6:42] - b[:, 6:42]), axis=1) / amp
        e_s = np.abs(a[:, 42] - b[:, 42]) / np.maximum(1.0, np.abs(b[:, 42]))
        cg, co = a[:, 43] + 1j * a[:, 44], b[:, 43] + 1j * b[:, 44]
        e_c = np.abs(cg - co) / np.maximum(1.0, np.abs(co)) / amp
        ratio = np.max(np.stack([e_qp, e_m, e_s, e_c]), axis=0) / tol
        reg = b[:, 46] <= M_REGULAR
        print(f"angle {P}: largest error / bound: regular {ratio[reg].max():.3e}, "
              f"max|M| > 1e4 {ratio[~reg].max():.3e} (median {np.median(ratio[~reg]):.3e})",
              flush=True)
        assert np.array_equal(a[reg, 45], b[reg, 45])
        assert np.all(ratio < 1.0), (P, live[np.argmax(ratio)], ratio.max())

"""The latency form of the FP64 trajectory kernel (one trajectory per 8
lanes, RK4 applied to each monodromy column on its own lane), through the C
ABI: against the oracle, against the one-trajectory-per-lane form on the
same trajectories, as the FP64 re-run of the mixed form, and in plans.

sfhk_propagate picks the form from the launch size (ceil(capacity / 64) +
n_prob <= 128 packs: latency form); an ensemble allocated with a larger
capacity than it holds runs the same trajectories in the other form.
"""
import math
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def sf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13686_amd as sf
    return sf


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_form(sf, probs, n, seeds, capacity, precision="fp64"):
    import torch
    ens = sf.Ensemble(capacity, len(probs))
    ens, ws = sf.sample_initial(probs, n, seeds, ens=ens)
    acc, fs = sf.propagate(probs, ens, precision, final_state=True, workspace=ws)
    torch.cuda.synchronize()
    return ens, acc.cpu().numpy(), fs.cpu().numpy()


@pytest.mark.parametrize("case", ["h2", "n2pair"])
def test_latency_form_matches_oracle_and_wide_form(sf, orc, case):
    if case == "h2":
        probs, n, seeds = [workloads.h2_softcore()], [4096], [1001]
    else:
        probs, n, seeds = [workloads.n2(0.0), workloads.n2(90.0)], [1500, 1500], [1002, 1002]
    print(f"latency form: {case} {n}", flush=True)
    ens, acc_l, fs_l = run_form(sf, probs, n, seeds, sum(n))           # <= 128 packs
    _, acc_w, fs_w = run_form(sf, probs, n, seeds, 200 * 64)           # > 128 packs
    offs, lens = sf.accum_layout(probs)
    w = ens.w.cpu().numpy()
    for P, (p, o, l) in enumerate(zip(probs, offs, lens)):
        acc_o, _, _ = orc.run(p, seeds[P], 0, n[P], NTHREADS)
        e_l, e_w = rel(acc_l[o:o + l], acc_o), rel(acc_w[o:o + l], acc_o)
        print(f"  problem {P}: dipole sum vs oracle: latency form {e_l:.2e}, wide form {e_w:.2e}",
              flush=True)
        assert e_l < 1e-10 and e_w < 1e-10
    # final records of every live slot: the two forms and the oracle
    live = np.nonzero(w[:sum(n)] > 0)[0]
    g = {f: getattr(ens, f).cpu().numpy() for f in ens.FIELDS_I32 + ens.FIELDS_F64}
    worst = 0.0
    rng = np.random.default_rng(5)
    for i in rng.choice(live, size=min(40, live.size), replace=False):
        p = probs[int(g["prob"][i])]
        _, fo = orc.trajectory(p, int(g["k0"][i]), (g["qx"][i], g["qy"][i], g["qz"][i]),
                               (g["px"][i], g["py"][i], g["pz"][i]),
                               (g["nx"][i], g["ny"][i], g["nz"][i]), g["w"][i], amplitudes=False)
        amp = 1.0 + fo[46]
        tol = 1e-12 * amp * math.sqrt(orc.n_steps(p) - int(g["k0"][i]) + 1)
        for fs in (fs_l, fs_w):
            a = fs[:, i]
            e = max(np.max(np.abs(a[0:6] - fo[0:6]) / np.maximum(1.0, np.abs(fo[0:6]))),
                    np.max(np.abs(a[6:42] - fo[6:42])) / amp,
                    abs(a[42] - fo[42]) / max(1.0, abs(fo[42])),
                    abs(a[46] - fo[46]) / fo[46])
            worst = max(worst, e / tol)
            assert e < tol, (i, e, tol)
            if fo[46] <= 1e4:
                assert a[45] == fo[45]
    # the count of recombination steps: the same gate on nearly equal states
    reg = live[fs_w[46, live] <= 1e4]
    tot_l, tot_w = fs_l[47, reg].sum(), fs_w[47, reg].sum()
    assert abs(tot_l - tot_w) <= 1e-4 * tot_w
    print(f"  final records vs oracle: largest error / bound {worst:.2e}", flush=True)


@pytest.mark.parametrize("case", ["h2", "n2pair", "n2cap"])
def test_pipelined_form_equals_one_wavefront_form(sf, orc, case):
    """Without records the latency form runs its orbit on a second wavefront
    a step ahead (pipelined); with records it runs on one wavefront.  Both
    take the same operations on the same operands: their dipole sums agree to
    the order of the atomics, and with the oracle to 1e-10."""
    import torch
    if case == "h2":
        probs, n, seeds = [workloads.h2_softcore()], [4096], [1001]
    elif case == "n2pair":
        probs, n, seeds = [workloads.n2(0.0), workloads.n2(90.0)], [1500, 1500], [1002, 1002]
    else:
        probs, n, seeds = [dict(workloads.n2(0.0), c_max=1e3)], [3000], [1002]
    print(f"pipelined vs one-wavefront latency form: {case} {n}", flush=True)
    ens, ws = sf.sample_initial(probs, n, seeds)
    acc_p, _ = sf.propagate(probs, ens, workspace=ws)                  # pipelined
    acc_1, _ = sf.propagate(probs, ens, final_state=True, workspace=ws)  # one wavefront
    torch.cuda.synchronize()
    acc_p, acc_1 = acc_p.cpu().numpy(), acc_1.cpu().numpy()
    offs, lens = sf.accum_layout(probs)
    for P, (p, o, l) in enumerate(zip(probs, offs, lens)):
        e1 = rel(acc_p[o:o + l], acc_1[o:o + l])
        acc_o, _, _ = orc.run(p, seeds[P], 0, n[P], NTHREADS)
        eo = rel(acc_p[o:o + l], acc_o)
        print(f"  problem {P}: pipelined vs one-wavefront {e1:.2e}, vs oracle {eo:.2e}", flush=True)
        assert e1 < 1e-13 and eo < 1e-10


def test_latency_form_prefactor_cap(sf, orc):
    """The prefactor cap in the latency form: the decision of a group's lane 0
    stops the whole trajectory (dipole sums against the oracle's with the
    same cap)."""
    import torch
    probs = [dict(workloads.n2(0.0), c_max=1e3), dict(workloads.h2_softcore(), c_max=100.0)]
    n, seeds = [3000, 2000], [1002, 1001]
    ens, ws = sf.sample_initial(probs, n, seeds)
    acc, _ = sf.propagate(probs, ens, workspace=ws)
    torch.cuda.synchronize()
    offs, lens = sf.accum_layout(probs)
    for P, (p, o, l) in enumerate(zip(probs, offs, lens)):
        acc_o, _, _ = orc.run(p, seeds[P], 0, n[P], NTHREADS)
        e = rel(acc[o:o + l].cpu().numpy(), acc_o)
        print(f"capped problem {P}: dipole sum vs oracle {e:.2e}", flush=True)
        assert e < 1e-10


def test_mixed_rerun_forms(sf):
    """The FP64 re-run of handed-over trajectories in both forms: a mixed plan
    with the latency re-run equals sfhk_propagate (which always re-runs in the
    latency form) to the order of the dipole atomics; with the strongly
    amplifying trajectories capped, the one-lane re-run agrees to 1e-9."""
    import torch
    probs = [workloads.n2(0.0), workloads.n2(90.0)]
    n, seeds = [8192, 8192], [1002, 1002]
    out = sf.run(probs, n, seeds, precision="mixed", h_max=1.0)
    torch.cuda.synchronize()
    pl = sf.Plan(probs, n, seeds, precision="mixed", tuning=(0, 8, 1, 1, 8), h_max=1.0)
    pl.run()
    torch.cuda.synchronize()
    k_ms, r_ms = pl.kernel_ms()
    print(f"mixed plan: kernel {k_ms:.2f} ms, latency-form re-run {r_ms:.2f} ms", flush=True)
    for i in range(2):
        assert rel(pl.v_of(i).cpu().numpy(), out["v"][i].cpu().numpy()) < 1e-12
    pl.close()
    capped = [dict(p, c_max=3e4) for p in probs]
    res = {}
    for lanes in (1, 8):
        for persistent in (0, 1):
            pl = sf.Plan(capped, n, seeds, precision="mixed", tuning=(persistent, 8, 1, 1, lanes),
                         h_max=1.0)
            pl.run()
            torch.cuda.synchronize()
            res[(lanes, persistent)] = [pl.v_of(i).cpu().numpy() for i in range(2)]
            pl.close()
    for key, v in res.items():
        for i in range(2):
            e = rel(v[i], res[(8, 0)][i])
            print(f"capped, re-run lanes {key[0]} persistent {key[1]}: vs latency per-pack {e:.2e}")
            assert e < 1e-9


def test_plan_rejects_bad_lane_count(sf):
    from paper_2608_13686_amd import SfhkError
    with pytest.raises(SfhkError):
        sf.Plan([workloads.h2_softcore()], [100], [1], tuning=(0, 8, 1, 1, 4))

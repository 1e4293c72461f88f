"""Benchmark of the SFHK hot path on one MI355X.

One step = the whole path over one batch: sample the ensemble, propagate
every live trajectory (RK4 + monodromy + action + HK prefactor +
recombination + dipole sum), normalise the dipole and take its harmonic
spectrum.  Headline workload (``value``): N2 (Eq. 7, Table I, eps^2 = 0.5)
at fixed alignment 0 and 90 degrees, 1200 nm / 1.5e14 W/cm^2 / 4-cycle
sin^2, dt = 0.05, 1,048,576 trajectories per angle, plain FP64 kernel.

``variants`` in the same line: the mixed-precision form on the same
trajectories (with its error against the FP64 run), the batched
H2 + N2 cos^4 workload over 64 lasers each (128 x 32,768 trajectories) as
one tuned persistent plan replayed from a HIP graph, and a seeded Poisson
stream of spectrum requests served with continuous batching (two policies)
beside a FIFO server that runs one request at a time on the plain FP64 path.

Prints one JSON line (metric, value, roofline, cpu_baseline, variants, ...).
"""
import argparse
import ctypes as C
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X: 256 CU x 4 SIMD x 16 FP64 FMA/clk x 2 x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector peak (packed FP32 issue)
M_REGULAR = 1e4                  # largest monodromy entry of a regular trajectory
N_PREFIX = 65536                 # trajectories per angle of the oracle comparison


def method_flops(prob):
    """Algorithmic flops of one trajectory-step as the method defines them
    (FMA = 2, transcendentals excluded), counted from the formulas: for the
    screened two-centre potential of Eq. 7, 4 potential/gradient/Hessian
    evaluations (116 flops each) and the -K M_q products (90), the RK4 stage
    algebra of all 43 components (602), the HK prefactor (111) and the phase
    and deposit (13): 1,580 flops, plus 340 for the recombination sum of the
    N2 orbital (4 s + 4 p primitives) at the steps that evaluate it; for the
    soft-core potential, 1,420 + 210 (6 s primitives).  Returns (stepping,
    fp64_fixed, recombination): the part the mixed form runs in FP32 (q, p,
    M, potential, det R) and the parts that stay FP64 (action, root of det R
    and branch, phase, amplitude, dipole; the recombination sum)."""
    screened = any(c["dZ"] != 0.0 for c in prob["target"]["centers"])
    gated = 1580 if screened else 1420
    recomb = 340 if screened else 210
    fp64_fixed = 130
    return gated - fp64_fixed, fp64_fixed, recomb


def flops_per_step(prob, f_near):
    """Method flops of one trajectory-step with the recombination sum counted
    at the fraction f_near of the steps at which the kernel evaluates it."""
    st, fx, rc = method_flops(prob)
    return st + fx + f_near * rc


def builder_flops_per_step(prob):
    """The earlier, larger count: RK4 of every monodromy column counted as
    textbook RK4 (972 flops) instead of the step matrix the kernel applies."""
    screened = any(c["dZ"] != 0.0 for c in prob["target"]["centers"])
    pot_centre = 60 if screened else 50
    return 4 * (2 * pot_centre + 9) + 92 + 6 * (4 * 18 + 3 * 24 + 18) + 121 + 16


def mixed_ceiling_steps_per_s(prob, f_near):
    """Upper bound of the mixed form's trajectory-steps/s: its FP32 part at the
    FP32 vector peak and its FP64 part at the FP64 vector peak, sharing the
    vector ALU."""
    st, fx, rc = method_flops(prob)
    t = st / (FP32_VECTOR_PEAK_TFLOPS * 1e12) + (fx + f_near * rc) / (FP64_VECTOR_PEAK_TFLOPS * 1e12)
    return 1.0 / t


def measured_traffic(kernel_file, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the kernel source as it is now; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel_file}__{workload}.traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2608_13686_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read()
                   for f in ("propagate_f64.hip", "device_common.h", "sfhk_internal.h"))
    if hashlib.sha256(src).hexdigest() != rec["kernel_sha256"]:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def near_fraction(sf, probs, n_traj, ens, ws):
    """Per problem, the fraction of a trajectory's steps at which the kernel
    evaluates the recombination sum (a shell of psi_0 passes its far-field
    cut), from the per-trajectory counts of an untimed run that keeps final
    records."""
    import torch
    _, fs = sf.propagate(probs, ens, final_state=True, workspace=ws)
    torch.cuda.synchronize()
    out, off = [], 0
    for p, n in zip(probs, n_traj):
        N = sf.problem_steps(p)[0]
        live = ens.w[off:off + n] > 0
        k0 = ens.k0[off:off + n].to(torch.float64)
        near = fs[sf.FS_NEAR, off:off + n]
        out.append(float(near[live].sum() / (N + 1 - k0[live]).sum()))
        off += n
    del fs
    torch.cuda.empty_cache()
    return out


def lscpu_model():
    try:
        import subprocess
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in r.stdout.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return cpu_model()


def cpu_baseline_and_parity(sf, probs, seeds):
    """The oracle on the first 65,536 trajectories of each problem of the
    headline workload, on the host's cores: its rate is the CPU baseline, and
    its dipole sums (all live trajectories, and the regular ones whose
    largest monodromy entry stays <= 1e4) are compared with the GPU's on the
    same trajectories (the GPU's regular sum zeroes the weights of the other
    slots)."""
    import oracle
    import torch
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    t = time.perf_counter()
    runs = [oracle.run_ensemble(p, s, 0, N_PREFIX, m_regular=M_REGULAR, nthreads=cores)
            for p, s in zip(probs, seeds)]
    el = time.perf_counter() - t
    steps = sum(r["live_steps"] for r in runs)
    print(f"oracle: {N_PREFIX} x {len(probs)} trajectories, {steps} live steps in {el:.1f} s "
          f"on {cores} cores", file=sys.stderr, flush=True)
    base = {"value": steps / el, "unit": "trajectory-steps/s", "cores": cores, "kind": "oracle",
            "per_core": steps / el / cores,
            "sample": f"trajectories 0..{N_PREFIX - 1} of each of the {len(probs)} problems of "
                      f"the headline workload ({steps} live trajectory-steps, {el:.1f} s; the "
                      f"same run gives the parity block)",
            "cpu_model": lscpu_model()}
    # the same trajectories on the GPU: every live one, then the regular ones only
    n = [N_PREFIX] * len(probs)
    ens, ws = sf.sample_initial(probs, n, seeds)
    acc_all, _ = sf.propagate(probs, ens, workspace=ws)
    chaotic = np.concatenate([r["finals"][:, oracle.F_MMAX] > M_REGULAR for r in runs])
    idx = torch.from_numpy(np.nonzero(chaotic)[0]).to(ens.w.device)
    ens.w[idx] = 0.0
    acc_reg, _ = sf.propagate(probs, ens, workspace=ws)
    torch.cuda.synchronize()
    offs, lens = sf.accum_layout(probs)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    per = []
    for P, (p, o, l, r) in enumerate(zip(probs, offs, lens, runs)):
        ga, gr = acc_all[o:o + l].cpu().numpy(), acc_reg[o:o + l].cpu().numpy()
        oa, orr = r["accum_all"], r["accum_regular"]
        m = r["finals"][:, oracle.F_MMAX]
        per.append({"theta_deg": round(math.degrees(p["align"]["theta"]), 3),
                    "live": int(r["n_live"]), "amplifying": int(np.sum(m > M_REGULAR)),
                    "largest_max_abs_M": float(m.max()),
                    "rel_l2_regular": rel(gr, orr), "rel_l2_all": rel(ga, oa),
                    "share_of_v_from_amplifying": rel(orr, oa),
                    "norm_regular_over_all": float(np.linalg.norm(orr) / np.linalg.norm(oa))})
    parity = {"workload": f"first {N_PREFIX} trajectories of each angle of the headline "
                          "workload, FP64 kernel vs oracle",
              "regular": f"largest |M_ij| along the trajectory <= {M_REGULAR:g} (oracle)",
              "tolerance_regular": 1e-10, "per_problem": per,
              "rel_l2_regular": max(x["rel_l2_regular"] for x in per),
              "rel_l2_all": max(x["rel_l2_all"] for x in per),
              "share_of_v_from_amplifying": min(x["share_of_v_from_amplifying"] for x in per)}
    del ens, ws, acc_all, acc_reg
    return base, parity


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def small_variant(sf, reps=5):
    """The small H2 workload (4,096 trajectories, 3,310 steps, harmonics to
    40) end to end: sampling, packing, propagation, dipole and spectrum.  At
    64 wavefronts on 1,024 SIMDs it measures latency, not throughput."""
    import torch
    p = workloads.h2_softcore()
    out = sf.run([p], [4096], [1001], h_max=40.0)  # warm-up
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        out = sf.run([p], [4096], [1001], h_max=40.0)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    ens, _ = sf.sample_initial([p], [4096], [1001])
    steps = live_steps_of(sf, [p], [4096], ens)
    best = min(ts)
    return {"workload": "h2-softcore-800nm-4096", "ms_per_run": best * 1e3,
            "ms_per_run_median": sorted(ts)[len(ts) // 2] * 1e3, "live_trajectory_steps": steps,
            "value": steps / best, "unit": "trajectory-steps/s", "precision": "fp64"}


def live_steps_of(sf, probs, n_traj, ens, per_problem=False):
    """Unit of work: sum over live trajectories of N - k0 (RK4 steps)."""
    import torch
    per, off = [], 0
    for p, n in zip(probs, n_traj):
        N = sf.problem_steps(p)[0]
        k0 = ens.k0[off:off + n].to(torch.int64)
        w = ens.w[off:off + n]
        per.append(int(((N - k0) * (w > 0)).sum().item()))
        off += n
    return per if per_problem else sum(per)


def plan_kernel_rooflines(plan, probs, live, f_near):
    """One untimed plan.run(), whose events time the trajectory kernel and
    the FP64 re-run on the plan's stream.  Kernel roofline: the method's
    flops over the live trajectory-steps; the FP64 kernel against the FP64
    vector peak, the mixed kernel against the mixed ceiling (FP32 part at the
    FP32 peak, FP64 part at the FP64 peak).  The re-run's work (about 1% of
    the trajectories, from their birth) is bounded by one wavefront's step
    latency, not by throughput: its time is reported as is."""
    import torch
    plan.run()
    torch.cuda.synchronize()
    k_ms, r_ms = plan.kernel_ms()
    steps = sum(live)
    flops = sum(n * flops_per_step(p, f) for n, p, f in zip(live, probs, f_near))
    out = {"kernel_ms": k_ms, "rerun_ms": r_ms, "live_trajectory_steps": steps,
           "f_near": [round(f, 5) for f in f_near]}
    if plan.precision == "fp64":
        ach = flops / (k_ms * 1e-3) / 1e12
        out["kernel_roofline"] = {"bound": "alu", "achieved": ach, "peak": FP64_VECTOR_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_PEAK_TFLOPS}
    else:
        t_min = sum(n / mixed_ceiling_steps_per_s(p, f) for n, p, f in zip(live, probs, f_near))
        out["kernel_roofline"] = {
            "bound": "alu", "achieved": steps / (k_ms * 1e-3), "peak": steps / t_min,
            "unit": "trajectory-steps/s", "frac": t_min / (k_ms * 1e-3),
            "peak_is": "FP32 part of the method flops at 157.3 TFLOP/s plus its FP64 part "
                       "at 78.6 TFLOP/s"}
    return out


def spectral_db(sf, prob, v_a, v_b, h_lo, h_hi):
    """Median and 90th percentile of |10 log10(Y_a / Y_b)| over H[h_lo, h_hi]."""
    import torch
    N, t0, tau = sf.problem_steps(prob)
    om = sf.harmonic_grid(prob, h_hi).cuda()
    _, ya = sf.spectrum(v_a, t0, prob["dt"], tau / 2, om)
    _, yb = sf.spectrum(v_b, t0, prob["dt"], tau / 2, om)
    h = torch.arange(om.numel(), dtype=torch.float64) * 0.05
    sel = (h >= h_lo) & (h <= h_hi)
    db = (10 * torch.log10(ya.cpu() / yb.cpu())).abs()[sel].numpy()
    return float(np.median(db)), float(np.percentile(db, 90))


_SIDE = None


def side_stream():
    """One side stream for every recorded graph: each extra stream takes a
    hardware queue of the process's few."""
    global _SIDE
    import torch
    if _SIDE is None:
        _SIDE = torch.cuda.Stream()
    return _SIDE


def timed_plan(sf, probs, n_traj, seeds, precision, tuning, steps, warmup, h_max):
    import torch
    plan = sf.Plan(probs, n_traj, seeds, precision=precision, tuning=tuning, h_max=h_max)
    side = side_stream()
    plan.capture(side)
    for _ in range(max(warmup, 1)):
        plan.replay(side)
    side.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        plan.replay(side)
    side.synchronize()
    el = time.perf_counter() - t
    return plan, el / steps


def chaos_cap(sf, p):
    """Prefactor cap for the error diagnostic: five times the free-spreading
    |C| = |1 - i gamma tau/2|^{3/2} of a trajectory that lives the whole
    pulse, so that regular trajectories stay below the mixed kernel's
    hand-over threshold (c_max/4) and only chaotic ones are cut."""
    _, _, tau = sf.problem_steps(p)
    return 5.0 * abs(1.0 - 0.5j * p["gamma"] * tau) ** 1.5


def batched_errors(sf, wb, tun, v_mixed):
    """Relative L2 of the mixed batched dipoles against an FP64 plan of the
    same trajectories (median and maximum over the problems), as run and with
    chaotic trajectories cut by the prefactor cap chaos_cap (the FP32
    stepping error of the regular ones)."""
    import torch

    def run(probs, precision):
        pl = sf.Plan(probs, wb["n_traj"], wb["seeds"], precision=precision, tuning=tun,
                     h_max=40.0)
        pl.run()
        torch.cuda.synchronize()
        out = [pl.v_of(i).clone() for i in range(len(probs))]
        pl.close()
        return out

    def summary(a, b):
        r = np.array([float(torch.linalg.norm(x - y) / torch.linalg.norm(y)) for x, y in zip(a, b)])
        return {"median": float(np.median(r)), "max": float(r.max()),
                "worst_problem": wb["problems"][int(r.argmax())]["name"]}

    res = {"rel_l2_vs_fp64": summary(v_mixed, run(wb["problems"], "fp64"))}
    capped = [dict(p, c_max=chaos_cap(sf, p)) for p in wb["problems"]]
    res["rel_l2_vs_fp64_chaos_cap"] = summary(run(capped, "mixed"), run(capped, "fp64"))
    res["chaos_cap"] = "5 |1 - i gamma tau/2|^1.5 per problem"
    return res


def saddle_variant(sf, n_traj, steps, warmup):
    """The headline N2 workload with births from the exact SFA saddle point:
    whole step (sampling + propagation + dipole + spectra) and the sampler's
    own time, both from HIP events on the stream the kernels run on."""
    import torch
    wl = workloads.workload_n2_fixed(n_traj)
    probs = [workloads.with_changes(p, ionization="saddle") for p in wl["problems"]]
    n, seeds = wl["n_traj"], wl["seeds"]
    stream = torch.cuda.current_stream()
    ens = sf.Ensemble(sum(n), len(probs))
    ens, ws = sf.sample_initial(probs, n, seeds, ens=ens)
    offs, lens = sf.accum_layout(probs)
    acc = torch.zeros(sum(lens), dtype=torch.float64, device="cuda")
    v = torch.empty_like(acc)
    grids = []
    for p in probs:
        N, t0, tau = sf.problem_steps(p)
        grids.append((t0, 0.5 * tau, sf.harmonic_grid(p, 100.0).cuda()))
    torch.cuda.synchronize()
    live = live_steps_of(sf, probs, n, ens)
    samp = []

    def step(timed):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sf.sample_initial(probs, n, seeds, ens=ens, workspace=ws)
        e1.record(stream)
        acc.zero_()
        sf.propagate(probs, ens, accum=acc, workspace=ws)
        sf.dipole(probs, acc, n, v_out=v)
        for (t0, tauh, om), o, l in zip(grids, offs, lens):
            sf.spectrum(v[o:o + l], t0, probs[0]["dt"], tauh, om)
        if timed:
            samp.append((e0, e1))

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t) / steps
    n_live = int((ens.w > 0).sum().item())
    return {"workload": wl["name"] + "-saddle", "value": live / sec, "unit": "trajectory-steps/s",
            "ms_per_step": sec * 1e3, "live_trajectory_steps": live, "live_trajectories": n_live,
            "sample_ms": float(np.mean([a.elapsed_time(b) for a, b in samp])),
            "precision": "fp64", "ionization": "saddle point of Eq. 2"}


def analysis_variant(sf, probs, ens, ws, v, offs, lens):
    """Time-frequency and return analysis of the headline ensemble: the
    Gabor map of each dipole (centres every 0.5 a.u. over the pulse,
    harmonics 0..100 in steps of 0.1, window 1/(3 w)) and the first classical
    return of every live trajectory (sphere of 8 a.u.), timed with HIP events."""
    import torch
    stream = torch.cuda.current_stream()
    res = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    n_pts = 0
    for p, o, l in zip(probs, offs, lens):
        N, t0, tau = sf.problem_steps(p)
        tc = torch.arange(-0.5 * tau, 0.5 * tau, 0.5, dtype=torch.float64)
        om = sf.harmonic_grid(p, 100.0, 0.1)
        sf.gabor(v[o:o + l], t0, p["dt"], sf.gabor_width(p), tc, om)
        n_pts += tc.numel() * om.numel()
    ev[1].record(stream)
    ev[2].record(stream)
    k_ret, e_ret = sf.return_steps(probs, ens, 8.0, workspace=ws)
    ev[3].record(stream)
    torch.cuda.synchronize()
    res["gabor_ms"] = ev[0].elapsed_time(ev[1])
    res["gabor_points"] = n_pts
    res["returns_ms"] = ev[2].elapsed_time(ev[3])
    res["returned_trajectories"] = int((k_ret >= 0).sum().item())
    res["live_trajectories"] = int((ens.w > 0).sum().item())
    return res


def averaging_study(sf, mol, ionization, sizes, reps, n_ref, cap=False):
    """Isotropic average of one molecule two ways at equal trajectory counts
    (Eq. 5 with ten fixed alignments at Gauss-Legendre nodes in cos(theta),
    each with N_s/10 trajectories, against the joint Monte Carlo over the
    axis of Eq. 6 with N_s trajectories), both against a joint run with n_ref
    trajectories.  ionization: "first_order" (an alignment-independent
    tunnelling weight) or "saddle" (the weight carries the axis-dependent
    ionisation matrix element of Eq. 1, the sampling weight of Eq. 6).  cap:
    every problem with the prefactor cap above free spreading, which cuts the
    strongly amplifying trajectories.  Per size: relative L2 error of the
    averaged dipole and median |dB| error of the yield at the odd harmonics
    5..33, root mean square over `reps` independent runs, and the trajectory
    ratio for equal dipole error, (err_standard / err_joint)^2."""
    import torch
    av = workloads.workload_averaging(mol, 10)
    probs_s, wts = av["standard"]
    joint = av["joint"]
    probs_s = [workloads.with_changes(p, ionization=ionization) for p in probs_s]
    joint = workloads.with_changes(joint, ionization=ionization)
    if cap:
        probs_s = [dict(p, c_max=chaos_cap(sf, p)) for p in probs_s]
        joint = dict(joint, c_max=chaos_cap(sf, joint))
    N, t0, tau = sf.problem_steps(joint)
    w0 = 45.56335252912 / joint["laser"]["lambda_nm"]
    om = torch.tensor([h * w0 for h in range(5, 35, 2)], dtype=torch.float64, device="cuda")

    def joint_v(n, seed):
        chunk, acc, done = 1 << 22, None, 0
        while done < n:
            m = min(chunk, n - done)
            out = sf.run([joint], [m], [seed], h_max=1.0)
            a = out["v"][0] * m
            acc = a if acc is None else acc + a
            done += m
            seed += 7919  # independent chunks
            del out
        return acc / n

    def standard_v(n, seed):
        m = max(n // len(probs_s), 1)
        out = sf.run(probs_s, [m] * len(probs_s), [seed * 31 + i for i in range(len(probs_s))],
                     h_max=1.0)
        return sum(w * v for w, v in zip(wts, out["v"]))

    def yield_of(v):
        _, Y = sf.spectrum(v, t0, joint["dt"], 0.5 * tau, om)
        return Y.cpu().numpy()

    t = time.perf_counter()
    ref = joint_v(n_ref, 999)
    ref_h, ref_y = ref.cpu().numpy(), yield_of(ref)
    norm = np.linalg.norm(ref_h)

    def errors(v):
        y = yield_of(v)
        return (np.linalg.norm(v.cpu().numpy() - ref_h) / norm,
                float(np.median(np.abs(10 * np.log10(y / ref_y)))))

    rows = []
    for n in sizes:
        ej = [errors(joint_v(n, 100 + r)) for r in range(reps)]
        es = [errors(standard_v(n, 200 + r)) for r in range(reps)]
        rms = lambda e, i: float(np.sqrt(np.mean([x[i] ** 2 for x in e])))
        rows.append({"n_traj": n, "rel_l2_joint": rms(ej, 0), "rel_l2_standard": rms(es, 0),
                     "odd_harmonic_db_joint": rms(ej, 1), "odd_harmonic_db_standard": rms(es, 1),
                     "trajectory_ratio": (rms(es, 0) / rms(ej, 0)) ** 2})
    torch.cuda.synchronize()
    return {"reference_trajectories": n_ref, "repetitions": reps, "rows": rows,
            "seconds": time.perf_counter() - t}


def averaging_variant(sf, sizes=(1 << 14, 1 << 16, 1 << 18, 1 << 20), reps=6):
    """The averaging study for H2 and N2, each with the first-order sampler
    and with the saddle-point sampler whose weight carries the axis-dependent
    ionisation element (the Eq. 6 weight), each as sampled and with the
    strongly amplifying trajectories cut by the prefactor cap (how much of the
    Monte Carlo error they carry)."""
    out = {"angles": [round(a, 3) for a in workloads.workload_averaging("H2")["thetas_deg"]]}
    for mol, n_ref in (("H2", 1 << 26), ("N2", 1 << 25)):
        for ion in ("first_order", "saddle"):
            for cap in (False, True):
                key = f"{mol}-{ion}" + ("-capped" if cap else "")
                out[key] = averaging_study(sf, mol, ion, sizes, reps, n_ref,
                                           cap)
                print(f"averaging {key}: {out[key]}", file=sys.stderr, flush=True)
    return out


def served_variant(sf, n_req, loads, h_max=100.0, h_step=0.1, n_sat=200):
    """Latency of a seeded Poisson stream of spectrum requests at fractions of
    the device's saturation rate, under continuous batching (shortest
    remaining work first, time-targeted windows) and under a FIFO server that
    runs one request at a time on the plain FP64 path, both live.

    Saturation: the first n_sat requests of the stream alone on the plain FP64
    path, back to back; saturation spectra/s = requests / their total time.
    The stream is drawn once at 1 request/s and its arrival times are scaled
    to each rate (same requests, same order)."""
    import torch
    from paper_2608_13686_amd.serve import (HipExecutor, Server, fifo_stream, latency_stats,
                                            plain_fp64_runner, serve_stream)
    n_omega = int(round(h_max / h_step)) + 1
    unit = workloads.request_stream(n_req, 1.0)
    runner = plain_fp64_runner(h_max, h_step)
    runner(unit[0][1], 4096, 1)  # warm-up
    t = time.perf_counter()
    for _, p, n, seed in unit[:n_sat]:
        runner(p, n, seed)
    svc = (time.perf_counter() - t) / min(n_sat, len(unit))
    sat = 1.0 / svc
    print(f"saturation {sat:.2f} spectra/s (mean service {1e3 * svc:.1f} ms over {n_sat})",
          file=sys.stderr, flush=True)
    pool = 48 << 30
    x = HipExecutor(pool, 64, n_omega, h_step)
    warm = Server(x, pool, max_requests=64)
    warm.submit("warm", unit[0][1], 4096, 1)
    warm.drain()
    torch.cuda.synchronize()

    def summary(done, t0, wall):
        st = latency_stats(done)
        span = max(r.finished for r in done) - t0
        return {"completed": len(done), "p50_s": st["p50_s"], "p99_s": st["p99_s"],
                "mean_s": st["mean_s"], "max_s": st["max_s"], "spectra_per_s": len(done) / span,
                "wall_s": wall}

    out = {"workload": f"poisson-{n_req}req-seed1004", "n_requests": n_req,
           "trajectories_total": int(sum(n for _, _, n, _ in unit)), "n_omega": n_omega,
           "precision": "fp64", "saturation_spectra_per_s": sat,
           "saturation_from": f"first {n_sat} requests back to back on the plain FP64 path",
           "served_policy": "srpt by estimated time left less 0.5 x waiting time, launches "
                            "filled to 8,192 wavefronts, windows of ~40 ms ending with the "
                            "shortest request of each launch (requests bound by their step "
                            "latency advance more steps), one window in flight; a request more "
                            "than one window behind its completion on a virtual FIFO server "
                            "runs alone to its end; a request alone runs its whole pulse in one "
                            "launch of the plain FP64 kernel",
           "loads": []}
    for load in loads:
        rate = load * sat
        stream = [(t / rate, p, n, seed) for (t, p, n, seed) in unit]
        S = Server(x, pool, max_requests=64)
        t = time.perf_counter()
        done = serve_stream(S, stream)
        res = {"load": load, "rate_hz": rate,
               "served_srpt": dict(summary(done, t, time.perf_counter() - t),
                                   peak_pool_bytes=S.peak_bytes, peak_concurrent=S.peak_active)}
        print(f"served at {load:g} x saturation ({rate:.2f}/s): {res['served_srpt']}",
              file=sys.stderr, flush=True)
        t = time.perf_counter()
        done = fifo_stream(stream, runner)
        res["fifo_fp64"] = summary(done, t, time.perf_counter() - t)
        print(f"fifo at {load:g} x saturation: {res['fifo_fp64']}", file=sys.stderr, flush=True)
        out["loads"].append(res)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-traj", type=int, default=1 << 20, help="trajectories per angle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (calibrates HBM counters)")
    ap.add_argument("--no-variants", action="store_true",
                    help="measure only the headline FP64 workload")
    ap.add_argument("--only", default="",
                    help="comma list of variants to run (mixed, batched, small, analysis, "
                         "saddle, averaging, served); default all")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-loads", default="0.5,0.8",
                    help="arrival rates as fractions of the measured saturation rate")
    args = ap.parse_args()
    only = {x for x in args.only.split(",") if x}
    unknown = only - {"mixed", "batched", "small", "analysis", "saddle", "averaging", "served"}
    if unknown:
        sys.exit(f"unknown variants: {sorted(unknown)}")
    if args.gpus != 1:
        print("bench.py measures one GPU: the path shards by trajectory index with one "
              "dipole reduction per problem, but only the single-GPU path is built; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2608_13686_amd as sf

    torch.cuda.set_device(0)
    if args.copy_mib > 0:
        a = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    wl = workloads.workload_n2_fixed(args.n_traj)
    probs, n_traj, seeds = wl["problems"], wl["n_traj"], wl["seeds"]
    stream = torch.cuda.current_stream()

    # buffers resident in HBM before timing
    total = sum(n_traj)
    ens = sf.Ensemble(total, len(probs))
    ens, ws = sf.sample_initial(probs, n_traj, seeds, ens=ens)
    offs, lens = sf.accum_layout(probs)
    acc = torch.zeros(sum(lens), dtype=torch.float64, device="cuda")
    v = torch.empty_like(acc)
    grids = []
    for p in probs:
        N, t0, tau = sf.problem_steps(p)
        grids.append((t0, 0.5 * tau, sf.harmonic_grid(p, 100.0).cuda()))
    torch.cuda.synchronize()
    # live trajectory-steps of this ensemble (unit of work): sum over live of N - k0
    live_per = live_steps_of(sf, probs, n_traj, ens, per_problem=True)
    live_steps = sum(live_per)

    prop_ms = []

    def step(timed):
        sf.sample_initial(probs, n_traj, seeds, ens=ens, workspace=ws)
        acc.zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sf.propagate(probs, ens, accum=acc, workspace=ws)
        e1.record(stream)
        sf.dipole(probs, acc, n_traj, v_out=v)
        for (t0, tauh, om), o, l in zip(grids, offs, lens):
            # Eq. 3 on the harmonic grid and on the zero-padded FFT grid
            sf.spectrum(v[o:o + l], t0, probs[0]["dt"], tauh, om)
            sf.spectrum_fft(v[o:o + l], t0, probs[0]["dt"], tauh)
        if timed:
            prop_ms.append((e0, e1))

    for _ in range(args.warmup):
        step(False)
        print(f"warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    kern_s = np.mean([a.elapsed_time(b) for a, b in prop_ms]) / 1e3
    print(f"timed {args.steps} steps in {el:.3f} s; propagate {kern_s * 1e3:.1f} ms/launch",
          file=sys.stderr, flush=True)

    # the method's flops per step need the fraction of steps that evaluate the
    # recombination sum, counted by an untimed run that keeps final records
    f_near = near_fraction(sf, probs, n_traj, ens, ws)
    algo_flops = sum(n * flops_per_step(p, f) for n, p, f in zip(live_per, probs, f_near))
    achieved = algo_flops / kern_s / 1e12
    traffic = measured_traffic("propagate_f64_kernel",
                               "n2_fixed_0_90_2x1048576") if args.n_traj == 1 << 20 else None
    # algorithmic bytes: each live trajectory's initial conditions and pack
    # index (96 B) read once, each problem's dipole (8 B per step) written once
    n_live = int((ens.w > 0).sum().item())
    algo_bytes = 96 * n_live + sum(8 * l for l in lens)
    out = {
        "metric": "HK trajectory-steps/s (FP64)",
        "value": live_steps * args.steps / el,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "problems": "N2 eq7 TableI eps2=0.5, theta 0 and 90 deg",
                   "laser": "1200nm 1.5e14Wcm2 4cyc sin2 cep0", "dt": 0.05,
                   "trajectories_per_problem": n_traj[0], "live_trajectory_steps": live_steps,
                   "precision": "fp64"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic,
                     "kernel": "propagate_f64_kernel", "kernel_ms": kern_s * 1e3,
                     "flops_per_traj_step": [round(flops_per_step(p, f), 1)
                                             for p, f in zip(probs, f_near)],
                     "flops_count": "1,580 per step + f_near x 340 for the recombination sum "
                                    "(N2, FMA = 2, transcendentals excluded)",
                     "f_near": [round(f, 5) for f in f_near],
                     "frac_with_builder_count_1717": builder_flops_per_step(probs[0]) *
                     live_steps / kern_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                     "algorithmic_bytes": algo_bytes,
                     "traffic_over_algorithmic_bytes": (traffic / algo_bytes) if traffic else None,
                     "traffic_gb_per_s": (traffic / kern_s / 1e9) if traffic else None},
    }
    if not args.no_variants:
        from paper_2608_13686_amd import autotune
        variants = {}
        def want(name):
            return not only or name in only
        if want("mixed"):
            # mixed precision on the same trajectories, error against the FP64 run
            v64 = v.clone()
            tun = autotune.cached(probs, "mixed") or (0, 8, 1, 1)
            plan, sec = timed_plan(sf, probs, n_traj, seeds, "mixed", tun, args.steps, args.warmup,
                                   100.0)
            errs_u = []
            for i, (p, o, l) in enumerate(zip(probs, offs, lens)):
                rel = float(torch.linalg.norm(plan.v_of(i) - v64[o:o + l]) /
                            torch.linalg.norm(v64[o:o + l]))
                errs_u.append({"theta_deg": round(math.degrees(p["align"]["theta"]), 3),
                               "rel_l2_vs_fp64": rel})
            kr = plan_kernel_rooflines(plan, probs, live_per, f_near)
            plan.close()
            del plan
            # the FP32 stepping error: the same comparison with the strongly
            # amplifying trajectories cut by a prefactor cap above free spreading
            capped = [dict(p, c_max=chaos_cap(sf, p)) for p in probs]
            errs_c = []
            pf = sf.Plan(capped, n_traj, seeds, precision="fp64", tuning=tun, h_max=100.0)
            pm = sf.Plan(capped, n_traj, seeds, precision="mixed", tuning=tun, h_max=100.0)
            pf.run()
            pm.run()
            torch.cuda.synchronize()
            for i, p in enumerate(capped):
                rel = float(torch.linalg.norm(pm.v_of(i) - pf.v_of(i)) / torch.linalg.norm(pf.v_of(i)))
                med, p90 = spectral_db(sf, p, pm.v_of(i), pf.v_of(i), 15.0, 80.0)
                errs_c.append({"theta_deg": round(math.degrees(p["align"]["theta"]), 3),
                               "c_max": p["c_max"], "rel_l2_vs_fp64": rel,
                               "spectral_db_median_H15_80": med,
                               "spectral_db_p90_H15_80": p90})
            pf.close()
            pm.close()
            del pf, pm
            variants["mixed"] = {
                "workload": wl["name"], "value": live_steps / sec,
                "unit": "trajectory-steps/s", "ms_per_step": sec * 1e3, "tuning": list(tun),
                "speedup_vs_fp64": (el / args.steps) / sec,
                "error_vs_fp64": errs_c,
                "error_is": "FP32 stepping error: both runs with the trajectories that amplify "
                            "rounding past the FP32 hand-over cut by the prefactor cap c_max",
                "error_vs_fp64_uncapped": errs_u,
                "error_uncapped_is": "not an FP32 error: the uncapped dipole is carried by the "
                                     "few strongly amplifying trajectories, which both runs "
                                     "propagate in FP64 (the mixed run hands them over)",
                **kr}
            print(f"mixed: {variants['mixed']}", file=sys.stderr, flush=True)
        if want("batched"):
            # batched cos^4 H2 + N2 over 64 lasers each, persistent plan, graph replay
            wb = workloads.workload_batched(32768)
            tun = autotune.cached(wb["problems"], wb["precision"]) or (1, 8, 1, 1)
            plan, sec = timed_plan(sf, wb["problems"], wb["n_traj"], wb["seeds"], wb["precision"],
                                   tun, args.steps, args.warmup, 40.0)
            per = live_steps_of(sf, wb["problems"], wb["n_traj"], plan.ens, per_problem=True)
            ls = sum(per)
            v_mixed = [plan.v_of(i).clone() for i in range(len(wb["problems"]))]
            ens_b, ws_b = sf.sample_initial(wb["problems"], wb["n_traj"], wb["seeds"])
            fb = near_fraction(sf, wb["problems"], wb["n_traj"], ens_b, ws_b)
            del ens_b, ws_b
            kr = plan_kernel_rooflines(plan, wb["problems"], per, fb)
            kr["f_near"] = {"median": float(np.median(fb)), "min": float(np.min(fb)),
                            "max": float(np.max(fb))}
            plan.close()
            del plan
            variants["batched"] = {"workload": wb["name"], "value": ls / sec,
                                   "unit": "trajectory-steps/s", "ms_per_step": sec * 1e3,
                                   "live_trajectory_steps": ls, "precision": wb["precision"],
                                   "tuning": list(tun), "launch": "one HIP graph per step",
                                   "error": batched_errors(sf, wb, tun, v_mixed), **kr}
            del v_mixed
            print(f"batched: {variants['batched']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        if want("small"):
            variants["small"] = small_variant(sf)
            print(f"small: {variants['small']}", file=sys.stderr, flush=True)
        if want("analysis"):
            variants["analysis"] = analysis_variant(sf, probs, ens, ws, v, offs, lens)
            print(f"analysis: {variants['analysis']}", file=sys.stderr, flush=True)
        if want("saddle"):
            variants["saddle"] = saddle_variant(sf, args.n_traj, args.steps, args.warmup)
            print(f"saddle: {variants['saddle']}", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        if want("averaging"):
            variants["averaging"] = averaging_variant(sf)
            print(f"averaging: {variants['averaging']}", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        if want("served") and args.serve_requests > 0:
            loads = [float(r) for r in str(args.serve_loads).split(",") if r]
            variants["served"] = served_variant(sf, args.serve_requests, loads)
        out["variants"] = variants
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity"] = cpu_baseline_and_parity(sf, probs, seeds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

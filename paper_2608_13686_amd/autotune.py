"""Autotuner of the plan launch options (sfhk_tuning).

Times a plan's recorded graph for each candidate (persistent queue or one
wavefront per pack, wavefronts per CU of the persistent grid, RK4 steps per
loop trip) on the workload it will serve, keeps the fastest, then, for the
mixed precision, times the fastest with the FP64 re-run of handed-over
trajectories in each form (1 lane per trajectory, or the 8-lane latency
form), and caches the choice as JSON per (GPU architecture, precision,
potential kinds, GTO primitives).  Trajectories per lane is fixed at 1: the
FP64 state of one trajectory already fills the register budget of two
wavefronts per SIMD, and two FP32 trajectories per lane would pay only
through packed FP32 arithmetic, which the library does not emit.

    python -m paper_2608_13686_amd.autotune --workload batched
"""
import argparse
import json
import os
import time

import torch

from . import Plan

CACHE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")

CANDIDATES = [(0, 8, u, 1, 8) for u in (1, 2, 4)] + [(1, w, u, 1, 8) for w in (4, 8, 12, 16)
                                                       for u in (1, 2, 4)]
RERUN_LANES = (1, 8)


def cache_key(probs, precision):
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    kinds = sorted({"screened" if any(c["dZ"] != 0 for c in p["target"]["centers"])
                    else "softcore" for p in probs})
    prims = sorted({len(p["target"]["gto"]) for p in probs})
    return f"{arch}_{precision}_{'+'.join(kinds)}_g{'-'.join(map(str, prims))}"


_SIDE = {}


def time_plan(probs, n_traj, seeds, precision, tuning, reps=2, h_max=40.0):
    plan = Plan(probs, n_traj, seeds, precision=precision, tuning=tuning, h_max=h_max)
    # one side stream for all candidates: each stream holds a hardware queue
    dev = torch.cuda.current_device()
    if dev not in _SIDE:
        _SIDE[dev] = torch.cuda.Stream()
    side = _SIDE[dev]
    plan.capture(side)
    plan.replay(side)  # warm-up
    side.synchronize()
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        plan.replay(side)
        side.synchronize()
        best = min(best, time.perf_counter() - t)
    plan.close()
    return best


def tune(probs, n_traj, seeds, precision, candidates=CANDIDATES, reps=2, verbose=True):
    rows = []
    for cand in candidates:
        t = time_plan(probs, n_traj, seeds, precision, cand, reps)
        rows.append({"tuning": list(cand), "seconds": t})
        if verbose:
            print(f"tuning {cand}: {t * 1e3:.1f} ms", flush=True)
    best = min(rows, key=lambda r: r["seconds"])
    if precision == "mixed":
        for lanes in RERUN_LANES:
            cand = tuple(best["tuning"][:4]) + (lanes,)
            if list(cand) == best["tuning"]:
                continue
            t = time_plan(probs, n_traj, seeds, precision, cand, reps)
            rows.append({"tuning": list(cand), "seconds": t})
            if verbose:
                print(f"tuning {cand}: {t * 1e3:.1f} ms", flush=True)
        best = min(rows, key=lambda r: r["seconds"])
    return {"key": cache_key(probs, precision), "best": best["tuning"], "table": rows,
            "workload": {"n_problems": len(probs), "n_traj": sum(n_traj)}}


def cached(probs, precision):
    """The cached best tuning for this kind of workload, or None."""
    path = os.path.join(CACHE_DIR, cache_key(probs, precision) + ".json")
    if not os.path.exists(path):
        return None
    best = tuple(json.load(open(path))["best"])
    return best if len(best) == 5 else best + (8,)  # choices kept before the lane knob


def save(result, out_dir=CACHE_DIR):
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, result["key"] + ".json")
    with open(path, "w") as f:
        json.dump(result, f, indent=1)
    return path


def main():
    import workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["batched", "n2"], default="batched")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None)
    ap.add_argument("--n-per-problem", type=int, default=None)
    ap.add_argument("--out-dir", default=CACHE_DIR)
    args = ap.parse_args()
    if args.workload == "batched":
        wl = workloads.workload_batched(args.n_per_problem or 32768)
    else:
        wl = workloads.workload_n2_fixed(args.n_per_problem or (1 << 20))
    prec = args.precision or wl["precision"]
    res = tune(wl["problems"], wl["n_traj"], wl["seeds"], prec)
    print(json.dumps({"key": res["key"], "best": res["best"]}), flush=True)
    print("saved", save(res, args.out_dir), flush=True)


if __name__ == "__main__":
    main()

"""Per-trajectory records of sfhk_propagate (final state and snapshots along
the pulse) and the single-buffer footprint of the path, through the C ABI.

Snapshots are checked against the oracle's trajectory stopped at the same
grid steps (q, p, M, S, the prefactor C with its branch, the running
maximum of |M|), against invariants at every snapshot of every regular
trajectory (det M = 1, |det R| >= 1, |C|^2 = |det R|), and for their
layout (steps before a trajectory's birth are left untouched).
"""
import ctypes as C
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13686_amd as sf
    return sf


def host(ens):
    return {f: getattr(ens, f).cpu().numpy() for f in ens.FIELDS_I32 + ens.FIELDS_F64}


def record_errors(a, b, k_steps):
    """Largest error of a GPU record a against an oracle record b, over the
    bound 1e-12 (1 + max|M|) sqrt(steps) used for final states."""
    amp = 1.0 + b[46]
    tol = 1e-12 * amp * math.sqrt(k_steps + 1)
    e = max(np.max(np.abs(a[0:6] - b[0:6]) / np.maximum(1.0, np.abs(b[0:6]))),
            np.max(np.abs(a[6:42] - b[6:42])) / amp,
            abs(a[42] - b[42]) / max(1.0, abs(b[42])),
            abs(complex(a[43], a[44]) - complex(b[43], b[44])) / max(1.0, abs(complex(b[43], b[44]))) / amp,
            abs(a[46] - b[46]) / b[46])
    return e / tol


def test_snapshots_match_oracle_and_invariants(sf, orc):
    import torch
    probs = [workloads.n2(30.0), workloads.h2_softcore()]
    n, seeds = [400, 600], [1002, 1001]
    every = 662  # divides the H2 grid (N = 3310), not the N2 one (N = 13238)
    Ns = [sf.problem_steps(p)[0] for p in probs]
    n_snap = max(Ns) // every + 1
    print(f"snapshots: N2 30 deg x 400 + H2 x 600, every {every} steps, {n_snap} snapshots",
          flush=True)
    ens, ws = sf.sample_initial(probs, n, seeds)
    acc, fs, snap = sf.propagate(probs, ens, final_state=True, snapshots=(n_snap, every),
                                 workspace=ws)
    acc0, _ = sf.propagate(probs, ens, workspace=ws)
    torch.cuda.synchronize()
    a, b = acc.cpu().numpy(), acc0.cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)  # records change no arithmetic
    g = host(ens)
    fs, snap = fs.cpu().numpy(), snap.cpu().numpy()
    steps = np.arange(n_snap) * every
    off = 0
    rng = np.random.default_rng(3)
    worst = 0.0
    for P, (p, nn, N) in enumerate(zip(probs, n, Ns)):
        sl = np.arange(off, off + nn)
        live = sl[g["w"][sl] > 0]
        dead = sl[g["w"][sl] == 0]
        # layout: records exactly at the steps k0 <= k <= N of live slots
        for i in live:
            has = np.isfinite(snap[:, 0, i])
            assert np.array_equal(has, (steps >= g["k0"][i]) & (steps <= N)), i
        assert np.all(np.isnan(snap[:, :, dead]))
        if N % every == 0:  # the last snapshot is the final state
            s_last = N // every
            assert np.array_equal(snap[s_last][:, live], fs[:, live])
        # invariants at every written snapshot of regular trajectories
        for s in range(n_snap):
            cols = live[np.isfinite(snap[s, 0, live])]
            rec = snap[s][:, cols]
            reg = rec[46] <= 1e4
            M = np.ascontiguousarray(rec[6:42, reg].T).reshape(-1, 6, 6)
            if M.shape[0] == 0:
                continue
            nm2 = np.linalg.norm(M, ord=2, axis=(1, 2)) ** 2
            gam = p["gamma"]
            R = 0.5 * (M[:, :3, :3] + M[:, 3:, 3:] - 1j * gam * M[:, :3, 3:] + 1j / gam * M[:, 3:, :3])
            dR = np.abs(np.linalg.det(R))
            Cabs2 = rec[43, reg] ** 2 + rec[44, reg] ** 2
            assert np.max(np.abs(np.linalg.det(M) - 1) / nm2) < 1e-7
            assert dR.min() >= 1 - 1e-6
            assert np.max(np.abs(Cabs2 - dR) / dR) < 1e-10
            assert np.all(rec[46, reg] >= np.max(np.abs(rec[6:42, reg]), axis=0))
        # against the oracle stopped at the snapshot steps
        for i in rng.choice(live, size=min(6, live.size), replace=False):
            k0 = int(g["k0"][i])
            q0, p0 = (g["qx"][i], g["qy"][i], g["qz"][i]), (g["px"][i], g["py"][i], g["pz"][i])
            nax = (g["nx"][i], g["ny"][i], g["nz"][i])
            _, _, Ck = orc.trajectory(p, k0, q0, p0, nax, g["w"][i], amplitudes=False,
                                      prefactors=True)
            for s in np.nonzero((steps >= k0) & (steps <= N))[0]:
                k = int(steps[s])
                _, fo = orc.trajectory(p, k0, q0, p0, nax, g["w"][i], k_end=k, amplitudes=False)
                r = record_errors(snap[s][:, i], fo, k - k0)
                worst = max(worst, r)
                assert r < 1.0, (P, i, k, r)
                assert snap[s][45, i] == fo[45]
                assert abs(complex(snap[s][43, i], snap[s][44, i]) - Ck[k]) <= \
                    1e-10 * (1.0 + fo[46]) ** 2 * abs(Ck[k])
        off += nn
    print(f"snapshots vs oracle: largest error / bound {worst:.3e}", flush=True)


def test_mixed_snapshots_of_handed_over_trajectories_are_fp64(sf):
    """A trajectory the mixed kernel hands to FP64 gets its records from the
    FP64 re-run: bit for bit those of the FP64 run (the count of
    recombination steps aside, which the re-run counts from its first
    deposit)."""
    import torch
    probs = [workloads.n2(0.0)]
    n, seeds = [3000], [1002]
    every = 500
    n_snap = sf.problem_steps(probs[0])[0] // every + 1
    ens, ws = sf.sample_initial(probs, n, seeds)
    _, f64, s64 = sf.propagate(probs, ens, "fp64", final_state=True,
                               snapshots=(n_snap, every), workspace=ws)
    _, fmx, smx = sf.propagate(probs, ens, "mixed", final_state=True,
                               snapshots=(n_snap, every), workspace=ws)
    torch.cuda.synchronize()
    f64, fmx, s64, smx = (x.cpu().numpy() for x in (f64, fmx, s64, smx))
    live = np.nonzero(ens.w.cpu().numpy() > 0)[0]
    handed = live[f64[46, live] > 3e4]  # surely past the FP32 hand-over bound 1e4
    assert handed.size > 0
    keep = [i for i in range(48) if i != 47]
    for i in handed:
        assert np.array_equal(fmx[keep, i], f64[keep, i])
        assert np.array_equal(smx[:, keep, i], s64[:, keep, i], equal_nan=True)
    # the others are FP32 records: close to FP64 but not equal
    reg = live[f64[46, live] < 3e3]  # (free spreading alone gives |M_qp| = t - t0, up to 660)
    e = np.max(np.abs(fmx[0:6, reg] - f64[0:6, reg]) / np.maximum(1, np.abs(f64[0:6, reg])))
    print(f"{handed.size} handed over; FP32 records of regular ones within {e:.2e}", flush=True)
    assert 0 < e < 1e-2


def _carve(buf, sizes):
    """256-byte aligned consecutive sub-buffers of a device byte buffer."""
    out, off = [], 0
    for nb in sizes:
        out.append(buf.data_ptr() + off)
        off += (nb + 255) & ~255
    return out, off


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_path_runs_in_its_footprint(sf, precision):
    """The whole path for one problem inside one buffer of
    sfhk_footprint_bytes: ensemble arrays, workspace, accum and v carved from
    it, every step called through the C ABI; the dipole equals the one of the
    standard path."""
    import torch
    from paper_2608_13686_amd import _abi
    L = _abi.lib()
    p = workloads.h2_softcore(20.0)
    n, seed = 5000, 1001
    N = sf.problem_steps(p)[0]
    fp = sf.footprint_bytes(p, n, precision)
    buf = torch.full((fp,), 0xAB, dtype=torch.uint8, device="cuda")
    arr = _abi.make_problems([p])
    ens_sizes = [4 * n, 4 * n] + [8 * n] * 11 + [4 * n, 4, 4, 8]
    ptrs, used = _carve(buf, ens_sizes)
    es = _abi.Ensemble()
    es.capacity = n
    names = ["k0", "prob", "qx", "qy", "qz", "px", "py", "pz", "w", "nx", "ny", "nz", "dph",
             "order", "live_start", "live_count", "pack_start"]
    for f, ptr in zip(names, ptrs):
        setattr(es, f, ptr)
    acc_v = 2 * ((8 * (N + 1) + 255) & ~255)
    ws_bytes = fp - used - acc_v
    assert ws_bytes > 0
    ws_ptr = buf.data_ptr() + used
    acc_ptr = ws_ptr + ws_bytes
    v_ptr = acc_ptr + ((8 * (N + 1) + 255) & ~255)
    assert v_ptr + 8 * (N + 1) <= buf.data_ptr() + fp
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    one = _abi.u64_array([n])
    _abi.check(L.sfhk_sample_initial(arr, 1, one, _abi.u64_array([seed]), _abi.u64_array([0]),
                                     C.byref(es), C.c_void_p(ws_ptr), ws_bytes, stream),
               "sample")
    buf[used + ws_bytes:used + ws_bytes + 8 * (N + 1)].zero_()  # the accumulator
    _abi.check(L.sfhk_propagate(arr, 1, C.byref(es), sf.PRECISION[precision],
                                C.c_void_p(acc_ptr), None, None, 0, 1, C.c_void_p(ws_ptr),
                                ws_bytes, stream), "propagate")
    _abi.check(L.sfhk_dipole(arr, 1, C.c_void_p(acc_ptr), one, C.c_void_p(v_ptr), stream),
               "dipole")
    # one byte less of workspace is refused before anything is enqueued
    assert L.sfhk_propagate(arr, 1, C.byref(es), sf.PRECISION[precision], C.c_void_p(acc_ptr),
                            None, None, 0, 1, C.c_void_p(ws_ptr), ws_bytes - 1, stream) == 2
    torch.cuda.synchronize()
    v = buf[v_ptr - buf.data_ptr():v_ptr - buf.data_ptr() + 8 * (N + 1)].view(torch.float64)
    ref = sf.run([p], [n], [seed], precision=precision)["v"][0]
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(v - ref) / torch.linalg.norm(ref))
    print(f"{precision}: footprint {fp} bytes for {n} trajectories; dipole rel L2 vs the "
          f"standard path {err:.2e}", flush=True)
    assert err < 1e-13

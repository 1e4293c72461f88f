"""Python binding of the MI355X SFHK hot path (``libsfhk.so``).

Argument marshalling only: torch tensors own the device memory, the current
torch stream is the HIP stream, and every step runs in the library's HIP
kernels.  The names follow the C ABI in ``include/sfhk.h``.
"""
import ctypes as C
import functools
import math

import torch

from . import _abi
from ._abi import (FS_COUNT, FS_CIM, FS_CRE, FS_FLIPS, FS_M, FS_MMAX, FS_NEAR, FS_P, FS_Q, FS_S,
                   SfhkError)

__all__ = ["problem_steps", "workspace_bytes", "footprint_bytes", "Ensemble", "sample_initial",
           "propagate", "dipole", "spectrum", "run", "SfhkError", "harmonic_grid", "abi_version",
           "Plan", "accum_layout", "gabor", "gabor_width", "return_steps"]

PRECISION = {"fp64": _abi.FP64, "mixed": _abi.MIXED}


def abi_version():
    return _abi.lib().sfhk_abi_version()


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _on_stream(fn):
    """Run a step on ``stream`` (if given): the stream first waits for the
    work already queued on torch's current stream (which made the inputs),
    and the step runs with ``stream`` as torch's current stream, so that the
    tensors it allocates, zeroes or combines are ordered with the library's
    kernels there.  The outputs are ready on ``stream``: a caller using them
    on another stream synchronises the two, as usual in torch."""
    @functools.wraps(fn)
    def wrapper(*args, stream=None, **kw):
        if stream is None:
            return fn(*args, **kw)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            return fn(*args, stream=stream, **kw)
    return wrapper


def problem_steps(prob):
    """(N, t_first, tau) of a problem dictionary."""
    arr = _abi.make_problems([prob])
    n, t0, tau = C.c_int32(), C.c_double(), C.c_double()
    _abi.check(_abi.lib().sfhk_problem_steps(arr, C.byref(n), C.byref(t0), C.byref(tau)),
               "sfhk_problem_steps")
    return n.value, t0.value, tau.value


def workspace_bytes(probs, capacity):
    arr = _abi.make_problems(probs)
    nb = _abi.lib().sfhk_workspace_bytes(arr, len(probs), int(capacity))
    if nb == 0:
        raise SfhkError(1, "sfhk_workspace_bytes")
    return nb


def footprint_bytes(prob, n_traj, precision="fp64"):
    """Device bytes of the whole path for one problem (sfhk_footprint_bytes)."""
    arr = _abi.make_problems([prob])
    nb = _abi.lib().sfhk_footprint_bytes(arr, int(n_traj), PRECISION[precision])
    if nb == 0:
        raise SfhkError(1, "sfhk_footprint_bytes")
    return nb


def accum_layout(probs):
    """(offsets, lengths) of each problem's segment in accum / v arrays."""
    offs, lens, o = [], [], 0
    for p in probs:
        n = problem_steps(p)[0] + 1
        offs.append(o)
        lens.append(n)
        o += n
    return offs, lens


class Ensemble:
    """Device structure of arrays of a sampled ensemble (see sfhk_ensemble)."""

    FIELDS_I32 = ("k0", "prob")
    FIELDS_F64 = ("qx", "qy", "qz", "px", "py", "pz", "w", "nx", "ny", "nz", "dph")

    def __init__(self, capacity, n_prob, device="cuda"):
        cap = max(int(capacity), 1)
        self.capacity = int(capacity)
        self.n_prob = int(n_prob)
        for f in self.FIELDS_I32:
            setattr(self, f, torch.empty(cap, dtype=torch.int32, device=device))
        for f in self.FIELDS_F64:
            setattr(self, f, torch.empty(cap, dtype=torch.float64, device=device))
        self.order = torch.empty(cap, dtype=torch.int32, device=device)
        self.live_start = torch.empty(n_prob, dtype=torch.int32, device=device)
        self.live_count = torch.empty(n_prob, dtype=torch.int32, device=device)
        self.pack_start = torch.empty(n_prob + 1, dtype=torch.int32, device=device)

    def struct(self):
        s = _abi.Ensemble()
        s.capacity = self.capacity
        for f in self.FIELDS_I32 + self.FIELDS_F64 + ("order", "live_start", "live_count",
                                                         "pack_start"):
            setattr(s, f, getattr(self, f).data_ptr())
        return s


@_on_stream
def sample_initial(probs, n_per_prob, seeds, first_index=None, ens=None, workspace=None,
                   stream=None, device="cuda"):
    """Sample and pack an ensemble; returns (Ensemble, workspace tensor)."""
    n_prob = len(probs)
    if first_index is None:
        first_index = [0] * n_prob
    total = sum(int(n) for n in n_per_prob)
    if ens is None:
        ens = Ensemble(total, n_prob, device)
    arr = _abi.make_problems(probs)
    nb = _abi.lib().sfhk_workspace_bytes(arr, n_prob, ens.capacity)
    if nb == 0:
        raise SfhkError(1, "sfhk_workspace_bytes")
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=device)
    es = ens.struct()
    _abi.check(_abi.lib().sfhk_sample_initial(
        arr, n_prob, _abi.u64_array(n_per_prob), _abi.u64_array(seeds),
        _abi.u64_array(first_index), C.byref(es), C.c_void_p(workspace.data_ptr()),
        workspace.numel(), _stream(stream)), "sfhk_sample_initial")
    return ens, workspace


@_on_stream
def propagate(probs, ens, precision="fp64", accum=None, final_state=False, workspace=None,
              snapshots=None, stream=None):
    """Propagate the ensemble and add sum_j Re a_jk into accum (created zeroed
    if None).  snapshots=(n_snap, snap_every) also records the state at the
    steps s snap_every, s < n_snap (a [n_snap, FS_COUNT, capacity] tensor
    filled with NaN where no record is written).  Returns (accum, final_state
    or None), or (accum, final_state, snapshots) when snapshots are asked for."""
    n_prob = len(probs)
    arr = _abi.make_problems(probs)
    dev = ens.k0.device
    if accum is None:
        n_acc = sum(accum_layout(probs)[1])
        accum = torch.zeros(n_acc, dtype=torch.float64, device=dev)
    nb = _abi.lib().sfhk_workspace_bytes(arr, n_prob, ens.capacity)
    if nb == 0:
        raise SfhkError(1, "sfhk_workspace_bytes")
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
    fs = None
    if final_state:
        fs = torch.zeros((FS_COUNT, max(ens.capacity, 1)), dtype=torch.float64, device=dev)
    snap, n_snap, every = None, 0, 1
    if snapshots is not None:
        n_snap, every = int(snapshots[0]), int(snapshots[1])
        snap = torch.full((max(n_snap, 1), FS_COUNT, max(ens.capacity, 1)), float("nan"),
                          dtype=torch.float64, device=dev)
    es = ens.struct()
    _abi.check(_abi.lib().sfhk_propagate(
        arr, n_prob, C.byref(es), PRECISION[precision], C.c_void_p(accum.data_ptr()),
        C.c_void_p(fs.data_ptr() if fs is not None else 0),
        C.c_void_p(snap.data_ptr() if snap is not None else 0), n_snap, every,
        C.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream)), "sfhk_propagate")
    if snapshots is not None:
        return accum, fs, snap
    return accum, fs


@_on_stream
def dipole(probs, accum, n_sampled, v_out=None, stream=None):
    """v_k = (2/N_s) accum_k per problem."""
    arr = _abi.make_problems(probs)
    if v_out is None:
        v_out = torch.empty_like(accum)
    _abi.check(_abi.lib().sfhk_dipole(arr, len(probs), C.c_void_p(accum.data_ptr()),
                                      _abi.u64_array(n_sampled), C.c_void_p(v_out.data_ptr()),
                                      _stream(stream)), "sfhk_dipole")
    return v_out


@_on_stream
def spectrum(v, t_first, dt, tau_H, omega, stream=None):
    """(V complex128 tensor, yield) of the Hanning-windowed transform (Eq. 3)."""
    v = v.contiguous()
    omega = omega.to(device=v.device, dtype=torch.float64).contiguous()
    n = omega.numel()
    Vr = torch.empty(n, dtype=torch.float64, device=v.device)
    Vi = torch.empty_like(Vr)
    Y = torch.empty_like(Vr)
    _abi.check(_abi.lib().sfhk_spectrum(
        C.c_void_p(v.data_ptr()), v.numel(), float(t_first), float(dt), float(tau_H),
        C.c_void_p(omega.data_ptr()), n, C.c_void_p(Vr.data_ptr()), C.c_void_p(Vi.data_ptr()),
        C.c_void_p(Y.data_ptr()), _stream(stream)), "sfhk_spectrum")
    return torch.complex(Vr, Vi), Y


@_on_stream
def spectrum_fft(v, t_first, dt, tau_H, log2_len=None, stream=None):
    """Eq. 3 on the grid w_j = 2 pi j / (L dt), j = 0 .. L/2, of a transform
    zero-padded to L = 2^log2_len (default: the power of two >= 8 n_t)
    (sfhk_spectrum_fft).  Returns (omega, V complex128, yield |A|^2, phase
    arg A) with A = -i w V the dipole acceleration's spectrum."""
    v = v.contiguous()
    n = v.numel()
    L_ = _abi.lib()
    b = L_.sfhk_fft_log2_len(n) if log2_len is None else int(log2_len)
    nb = L_.sfhk_spectrum_fft_work_bytes(b)
    if nb == 0:
        raise SfhkError(1, "sfhk_spectrum_fft_work_bytes")
    work = torch.empty(nb, dtype=torch.uint8, device=v.device)
    m = (1 << b) // 2 + 1
    Vr = torch.empty(m, dtype=torch.float64, device=v.device)
    Vi, Y, ph = torch.empty_like(Vr), torch.empty_like(Vr), torch.empty_like(Vr)
    _abi.check(L_.sfhk_spectrum_fft(
        C.c_void_p(v.data_ptr()), n, float(t_first), float(dt), float(tau_H), b,
        C.c_void_p(work.data_ptr()), nb, C.c_void_p(Vr.data_ptr()), C.c_void_p(Vi.data_ptr()),
        C.c_void_p(Y.data_ptr()), C.c_void_p(ph.data_ptr()), _stream(stream)), "sfhk_spectrum_fft")
    omega = 2.0 * math.pi * torch.arange(m, dtype=torch.float64, device=v.device) / ((1 << b) * dt)
    return omega, torch.complex(Vr, Vi), Y, ph


@_on_stream
def acceleration(v, t_first, dt, tau_H, log2_len=None, stream=None):
    """The dipole acceleration on the step grid: the time derivative of the
    windowed dipole through its zero-padded spectrum (sfhk_acceleration)."""
    v = v.contiguous()
    n = v.numel()
    L_ = _abi.lib()
    b = L_.sfhk_fft_log2_len(n) if log2_len is None else int(log2_len)
    nb = L_.sfhk_spectrum_fft_work_bytes(b)
    if nb == 0:
        raise SfhkError(1, "sfhk_spectrum_fft_work_bytes")
    work = torch.empty(nb, dtype=torch.uint8, device=v.device)
    a = torch.empty(n, dtype=torch.float64, device=v.device)
    _abi.check(L_.sfhk_acceleration(
        C.c_void_p(v.data_ptr()), n, float(t_first), float(dt), float(tau_H), b,
        C.c_void_p(work.data_ptr()), nb, C.c_void_p(a.data_ptr()), _stream(stream)),
        "sfhk_acceleration")
    return a


@_on_stream
def return_steps(probs, ens, r_return=4.0, workspace=None, stream=None):
    """(k_ret int32, e_ret) per slot: first return step into |q| < r_return
    (-1 if none) and the kinetic energy there (sfhk_return_steps)."""
    arr = _abi.make_problems(probs)
    dev = ens.k0.device
    nb = _abi.lib().sfhk_workspace_bytes(arr, len(probs), ens.capacity)
    if nb == 0:
        raise SfhkError(1, "sfhk_workspace_bytes")
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
    cap = max(ens.capacity, 1)
    k_ret = torch.empty(cap, dtype=torch.int32, device=dev)
    e_ret = torch.empty(cap, dtype=torch.float64, device=dev)
    es = ens.struct()
    _abi.check(_abi.lib().sfhk_return_steps(
        arr, len(probs), C.byref(es), float(r_return), C.c_void_p(k_ret.data_ptr()),
        C.c_void_p(e_ret.data_ptr()), C.c_void_p(workspace.data_ptr()), workspace.numel(),
        _stream(stream)), "sfhk_return_steps")
    return k_ret, e_ret


@_on_stream
def gabor(v, t_first, dt, sigma, t_c, omega, stream=None):
    """(G complex128 [n_c, n_omega], yield) of the Gaussian-window transform
    (sfhk_gabor) of v at window centres t_c and frequencies omega."""
    v = v.contiguous()
    tc = torch.as_tensor(t_c, dtype=torch.float64).to(v.device).contiguous()
    om = torch.as_tensor(omega, dtype=torch.float64).to(v.device).contiguous()
    Gr = torch.empty((tc.numel(), om.numel()), dtype=torch.float64, device=v.device)
    Gi = torch.empty_like(Gr)
    Y = torch.empty_like(Gr)
    _abi.check(_abi.lib().sfhk_gabor(
        C.c_void_p(v.data_ptr()), v.numel(), float(t_first), float(dt), float(sigma),
        C.c_void_p(tc.data_ptr()), tc.numel(), C.c_void_p(om.data_ptr()), om.numel(),
        C.c_void_p(Gr.data_ptr()), C.c_void_p(Gi.data_ptr()), C.c_void_p(Y.data_ptr()),
        _stream(stream)), "sfhk_gabor")
    return torch.complex(Gr, Gi), Y


def gabor_width(prob):
    """Default Gabor window width 1/(3 w_laser) of a problem."""
    return prob["laser"]["lambda_nm"] / (3.0 * 45.56335252912)


def harmonic_grid(prob, h_max, h_step=0.05):
    """omega on the harmonic grid h = 0:h_step:h_max of the problem's laser."""
    omega0 = 45.56335252912 / prob["laser"]["lambda_nm"]
    n = int(round(h_max / h_step)) + 1
    return torch.arange(n, dtype=torch.float64) * h_step * omega0


@_on_stream
def run(probs, n_traj, seeds, precision="fp64", h_max=40.0, h_step=0.05, device="cuda",
        stream=None):
    """Whole path for a list of problems: sample, propagate, dipole and the
    spectrum of each problem on its harmonic grid.  Returns a dict."""
    ens, ws = sample_initial(probs, n_traj, seeds, device=device, stream=stream)
    acc, _ = propagate(probs, ens, precision, workspace=ws, stream=stream)
    v = dipole(probs, acc, n_traj, stream=stream)
    offs, lens = accum_layout(probs)
    out = {"v": [], "V": [], "yield": [], "omega": [], "t_first": [], "ensemble": ens}
    for p, o, n in zip(probs, offs, lens):
        N, t0, tau = problem_steps(p)
        om = harmonic_grid(p, h_max, h_step).to(device)
        V, Y = spectrum(v[o:o + n], t0, p["dt"], 0.5 * tau, om, stream=stream)
        out["v"].append(v[o:o + n])
        out["V"].append(V)
        out["yield"].append(Y)
        out["omega"].append(om)
        out["t_first"].append(t0)
    return out


class Plan:
    """The whole path for a batch of problems behind one plan (sfhk_plan_*):
    ``run()`` enqueues sampling, packing, propagation, dipole and spectra;
    ``capture(stream)`` records the same into a HIP graph that ``replay()``
    launches.  Outputs (overwritten by every run): ``accum``, ``v`` (accum
    layout), ``V`` and ``yield_`` ([n_prob, n_omega] on each problem's
    harmonic grid h = 0, h_step, ..., h_max)."""

    def __init__(self, probs, n_traj, seeds, precision="fp64", tuning=None, h_max=40.0,
                 h_step=0.05, first_index=None, device="cuda", stream=None):
        self.probs = list(probs)
        self.precision = precision
        n_prob = len(self.probs)
        self.n_traj = [int(n) for n in n_traj]
        self.first_index = [0] * n_prob if first_index is None else list(first_index)
        self.n_omega = int(round(h_max / h_step)) + 1
        self.h_step = h_step
        self._arr = _abi.make_problems(self.probs)
        L = _abi.lib()
        nb = L.sfhk_plan_workspace_bytes(self._arr, n_prob, _abi.u64_array(self.n_traj))
        if nb == 0:
            raise SfhkError(1, "sfhk_plan_workspace_bytes")
        self.ens = Ensemble(sum(self.n_traj), n_prob, device)
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=device)
        self.offsets, self.lengths = accum_layout(self.probs)
        n_acc = sum(self.lengths)
        self.accum = torch.zeros(n_acc, dtype=torch.float64, device=device)
        self.v = torch.zeros(n_acc, dtype=torch.float64, device=device)
        self.V_re = torch.zeros((n_prob, self.n_omega), dtype=torch.float64, device=device)
        self.V_im = torch.zeros_like(self.V_re)
        self.yield_ = torch.zeros_like(self.V_re)
        t = _abi.Tuning(*(tuning or (0, 8, 1, 1)))
        es = self.ens.struct()
        h = C.c_void_p()
        self._streams = set()
        _abi.check(L.sfhk_plan_create(
            self._arr, n_prob, _abi.u64_array(self.n_traj), _abi.u64_array(seeds),
            _abi.u64_array(self.first_index), PRECISION[precision], C.byref(t), float(h_step),
            self.n_omega, C.byref(es), C.c_void_p(self.workspace.data_ptr()),
            self.workspace.numel(), C.c_void_p(self.accum.data_ptr()),
            C.c_void_p(self.v.data_ptr()), C.c_void_p(self.V_re.data_ptr()),
            C.c_void_p(self.V_im.data_ptr()), C.c_void_p(self.yield_.data_ptr()),
            self._on(stream), C.byref(h)), "sfhk_plan_create")
        self._h = h

    def _buffers(self):
        yield from (getattr(self.ens, f) for f in self.ens.FIELDS_I32 + self.ens.FIELDS_F64 +
                    ("order", "live_start", "live_count", "pack_start"))
        yield from (self.workspace, self.accum, self.v, self.V_re, self.V_im, self.yield_)

    def _on(self, stream):
        """The plan's buffers are allocated and initialised on the current
        stream: work on another stream first waits for the current stream,
        and is recorded with the allocator, so that freeing the plan while
        that work is in flight cannot hand its memory to a new tensor."""
        cur = torch.cuda.current_stream()
        if stream is not None and stream != cur:
            stream.wait_stream(cur)
            if stream.cuda_stream not in self._streams:
                for t in self._buffers():
                    t.record_stream(stream)
                self._streams.add(stream.cuda_stream)
        return _stream(stream)

    def run(self, stream=None):
        _abi.check(_abi.lib().sfhk_plan_run(self._h, self._on(stream)), "sfhk_plan_run")

    def capture(self, stream):
        """Record run() into a HIP graph on a non-default torch stream."""
        _abi.check(_abi.lib().sfhk_plan_capture(self._h, self._on(stream)), "sfhk_plan_capture")

    def replay(self, stream=None):
        _abi.check(_abi.lib().sfhk_plan_replay(self._h, self._on(stream)), "sfhk_plan_replay")

    def kernel_ms(self):
        """(trajectory kernel, FP64 re-run) durations in ms of the last run()
        (HIP events on its stream; 0 for the re-run of an FP64 plan)."""
        ms = (C.c_float * 2)()
        _abi.check(_abi.lib().sfhk_plan_kernel_ms(self._h, ms), "sfhk_plan_kernel_ms")
        return ms[0], ms[1]

    @property
    def V(self):
        return torch.complex(self.V_re, self.V_im)

    def v_of(self, i):
        return self.v[self.offsets[i]:self.offsets[i] + self.lengths[i]]

    def omega(self, i):
        return harmonic_grid(self.probs[i], (self.n_omega - 1) * self.h_step, self.h_step)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _abi.lib().sfhk_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

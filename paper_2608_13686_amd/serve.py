"""Continuous-batching server of HHG-spectrum requests.

Requests (one problem, a trajectory count and a seed each) are admitted by
their device-memory footprint into a caller-sized pool and a slot of the
device request table; every scheduling step launches one window of RK4
steps over all admitted requests (``sfhk_serve_window``), so that requests
arriving while others run join at the next window and their work overlaps on
the device.  A request whose windows cover its whole pulse is finalised
(dipole + spectrum), its result copied out and its memory released.

The scheduling logic runs against an executor: ``HipExecutor`` drives the
HIP library; the tests drive the same scheduler with a host-only executor.
"""
import ctypes as C
import math
import time
from collections import deque

from . import _abi

ALIGN = 256


class PoolAllocator:
    """First-fit allocator of byte ranges in [0, size) with 256-byte
    alignment; freed ranges are coalesced with their neighbours."""

    def __init__(self, size, align=ALIGN):
        self.size = int(size)
        self.align = align
        self.free_list = [(0, self.size)]  # sorted (offset, length)
        self.used = {}

    def _round(self, n):
        return (int(n) + self.align - 1) // self.align * self.align

    def alloc(self, nbytes):
        n = self._round(max(nbytes, 1))
        for i, (off, ln) in enumerate(self.free_list):
            if ln >= n:
                if ln == n:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + n, ln - n)
                self.used[off] = n
                return off
        return None

    def free(self, off):
        n = self.used.pop(off)
        fl = self.free_list
        fl.append((off, n))
        fl.sort()
        merged = []
        for o, ln in fl:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free_list = merged

    @property
    def bytes_used(self):
        return sum(self.used.values())

    def largest_free(self):
        return max((ln for _, ln in self.free_list), default=0)


class Request:
    def __init__(self, tag, problem, n_traj, seed, arrival, deadline=None):
        self.tag = tag
        self.deadline = deadline
        self.error = None
        self.problem = problem
        self.n_traj = int(n_traj)
        self.seed = int(seed)
        self.arrival = arrival
        self.admitted = None
        self.finished = None
        self.slot = None
        self.offset = None
        self.bytes = None
        self.n_steps = None
        self.k_next = 0
        self.fifo_finish = None  # completion on a virtual FIFO server (seconds)
        self.handle = None
        self.event = None
        self.result = None
        self.host_result = None
        self.state = "waiting"


class HipExecutor:
    """Device side of the server: a torch uint8 pool, the request table and
    the C ABI calls.  Requests are sampled and finalised on the main stream;
    their packs can be split into `n_groups` interleaved groups, each advanced
    by its own stream (group 0 by the main stream itself), so that the tail
    of one group's window overlaps the others' windows.  All streams have the
    default priority.  One group is the default: a lone request split over
    two streams ran 1.3-1.4x slower than in one (measured on requests of
    1e5-2e5 trajectories); the streams need hardware queues of their own (a
    process has 4 by default) for any overlap to happen."""

    def __init__(self, pool_bytes, max_requests, n_omega, h_step, device="cuda", stream=None,
                 n_groups=1):
        import torch
        self.torch = torch
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        nb = _abi.lib().sfhk_request_table_bytes(max_requests)
        self.table = torch.empty(nb, dtype=torch.uint8, device=device)
        self.max_requests = max_requests
        self.n_omega = n_omega
        self.h_step = h_step
        self.stream = stream or torch.cuda.current_stream()
        self._h = C.c_void_p(self.stream.cuda_stream)
        self.n_groups = int(n_groups)
        self.group_streams = [self.stream] + [torch.cuda.Stream(device=device)
                                              for _ in range(self.n_groups - 1)]
        # the pool and the table are allocated on the current stream: work on
        # the other streams is recorded with the allocator, so that dropping
        # the executor while a window is in flight cannot reuse their memory
        for gs in self.group_streams:
            if gs != torch.cuda.current_stream():
                self.pool.record_stream(gs)
                self.table.record_stream(gs)

    def footprint(self, problem, n_traj):
        arr = _abi.make_problems([problem])
        nb = _abi.lib().sfhk_request_bytes(arr, int(n_traj), self.n_omega)
        if nb == 0:
            raise _abi.SfhkError(1, "sfhk_request_bytes")
        return nb

    def steps(self, problem):
        from . import problem_steps
        return problem_steps(problem)[0]

    def _event(self, stream):
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def init(self, req):
        req.handle = arr = _abi.make_problems([req.problem])
        _abi.check(_abi.lib().sfhk_request_init(
            arr, req.n_traj, req.seed, 0, float(self.h_step), self.n_omega,
            C.c_void_p(self.pool.data_ptr() + req.offset), req.bytes,
            C.c_void_p(self.table.data_ptr()), self.max_requests, req.slot, self._h),
            "sfhk_request_init")
        ev = self._event(self.stream)
        for gs in self.group_streams[1:]:
            gs.wait_event(ev)

    def window(self, entries, group=0):
        """entries: list of (request, k_from, k_to); advances pack group `group`.
        A lone request's window over its whole pulse runs the plain FP64
        kernel of sfhk_propagate (sfhk_request_run): no state is kept
        between windows it does not have."""
        n = len(entries)
        if n == 1 and self.n_groups == 1:
            r, k_from, k_to = entries[0]
            if k_from == 0 and k_to == r.n_steps + 1:
                _abi.check(_abi.lib().sfhk_request_run(
                    r.handle, r.n_traj, self.n_omega, C.c_void_p(self.pool.data_ptr() + r.offset),
                    r.bytes, C.c_void_p(self.table.data_ptr()), self.max_requests, r.slot,
                    self._h), "sfhk_request_run")
                return self._event(self.stream)
        slots = (C.c_int32 * n)(*[r.slot for r, _, _ in entries])
        ntraj = (C.c_uint64 * n)(*[r.n_traj for r, _, _ in entries])
        kf = (C.c_int32 * n)(*[a for _, a, _ in entries])
        kt = (C.c_int32 * n)(*[b for _, _, b in entries])
        gs = self.group_streams[group]
        _abi.check(_abi.lib().sfhk_serve_window(C.c_void_p(self.table.data_ptr()),
                                                self.max_requests, n, slots, ntraj, kf, kt,
                                                group, self.n_groups,
                                                C.c_void_p(gs.cuda_stream)), "sfhk_serve_window")
        return self._event(gs)

    def finalize(self, req):
        """Enqueues the request's dipole and spectrum and the copies of its
        results into pinned host memory, right behind its last window (ahead
        of any window queued later); the returned event marks the results
        ready on the host."""
        torch = self.torch
        for gs in self.group_streams[1:]:
            self.stream.wait_event(self._event(gs))
        _abi.check(_abi.lib().sfhk_request_finalize(
            req.handle, self.n_omega, C.c_void_p(self.table.data_ptr()),
            self.max_requests, req.slot, self._h), "sfhk_request_finalize")
        offs = (C.c_size_t * 4)()
        _abi.check(_abi.lib().sfhk_request_layout(req.handle, req.n_traj, self.n_omega, offs),
                   "sfhk_request_layout")
        base = req.offset
        sizes = {"v": req.n_steps + 1, "V_re": self.n_omega, "V_im": self.n_omega,
                 "yield": self.n_omega}
        host = {}
        with torch.cuda.stream(self.stream):
            for (name, n), off in zip(sizes.items(), offs):
                dev = self.pool[base + off: base + off + 8 * n].view(torch.float64)
                host[name] = torch.empty(n, dtype=torch.float64, pin_memory=True)
                host[name].copy_(dev, non_blocking=True)
        req.host_result = host
        return self._event(self.stream)

    def retire(self, req):
        """Event after which no queued work touches the request's memory."""
        for gs in self.group_streams[1:]:
            self.stream.wait_event(self._event(gs))
        return self._event(self.stream)

    def done(self, ev):
        return ev.query()

    def wait(self, ev):
        ev.synchronize()

    def result(self, req):
        """The results copied by finalize (valid once its event is done)."""
        out = req.host_result
        req.host_result = None
        return out


class Server:
    """Admission by footprint and table slots; every scheduling step launches
    one window of `window` RK4 steps for the requests it picks, with at most
    `in_flight` launches queued on the device.

    Policies: ``"ps"`` advances every admitted request each step (processor
    sharing); ``"srpt"`` advances first the requests with the least
    estimated time left alone on the device (`time_left_us`) less
    `age_weight` x their waiting time, so that short requests overtake long
    ones and a long one that has waited long enough goes first; it adds
    requests until the launch holds at least `fill_waves` wavefronts (default:
    4 x the `device_waves` the device keeps resident), so the device stays
    full.  With `fifo_bound` (default) each request also has a completion
    time on a virtual FIFO server (one request at a time in arrival order,
    each taking its fitted time alone: est_overhead_us + max(est_step_us,
    n x est_traj_step_us) per step); a request that would finish more than
    one window after it runs alone to the end of its pulse, so that the
    large requests a size-ordered policy delays are held near their FIFO
    latency.  ``"backfill"`` always runs the oldest request and fills with the
    others by least remaining work; ``"deadline"`` runs earliest arrival +
    `slack` x (estimated time alone) first.  Measured on a Poisson stream of
    1,000 mixed H2/N2 requests at 0.5 and 0.8 of the saturation rate: a fill
    of 2,048 wavefronts doubled srpt's p99 at 0.8; aging (age_weight 0.5)
    took p99 at 0.8 from 510 to 474 ms; one window in flight (in_flight=1:
    an arrival waits for at most the running window) took p50 at 0.5 from
    49 to 47 ms; backfill and deadline trailed srpt.

    Window length.  With `window_ms` (the default), a window lasts about
    `window_ms`: `window_ms / t_step` steps, where one step of a launch of n
    trajectories takes t_step = max(step_us, n x traj_step_us) (a launch
    below ~6,000 wavefronts is bound by one wavefront's step latency, a larger
    one by throughput: measured ~3 us and ~1e-5 us per trajectory-step), at
    least `window` steps, and no longer than the shortest picked request
    needs, so that it is finalised as soon as its pulse ends; a request
    running alone with nothing waiting runs to the end of its pulse in one
    window, the plain FP64 kernel (every window boundary re-synchronises all
    of its wavefronts and saves and restores 376 B per trajectory).  With window_ms=None every window is `window`
    steps, stretched up to `max_stretch` times for launches with fewer
    wavefronts than the device keeps resident (`device_waves`, 2 per SIMD on
    1,024 SIMDs)."""

    def __init__(self, executor, pool_bytes, max_requests=64, window=1024, in_flight=1,
                 policy="srpt", fill_waves=None, device_waves=2048, max_stretch=8,
                 window_ms=40.0, step_us=4.0, traj_step_us=1e-5, slack=4.0, age_weight=0.5,
                 fifo_bound=True, est_overhead_us=2500.0, est_step_us=2.7,
                 est_traj_step_us=9.4e-6, clock=time.perf_counter):
        if policy not in ("ps", "srpt", "backfill", "deadline"):
            raise ValueError("policy must be 'ps', 'srpt', 'backfill' or 'deadline'")
        if window < 1 or in_flight < 1 or max_requests < 1:
            raise ValueError("window, in_flight and max_requests must be positive")
        self.x = executor
        self.alloc = PoolAllocator(pool_bytes)
        self.free_slots = deque(range(max_requests))
        self.window = int(window)
        self.in_flight = in_flight
        self.policy = policy
        self.device_waves = int(device_waves)
        self.fill_waves = 4 * self.device_waves if fill_waves is None else int(fill_waves)
        self.max_stretch = max(1, int(max_stretch))
        self.window_ms = None if window_ms is None else float(window_ms)
        self.step_us = float(step_us)
        self.traj_step_us = float(traj_step_us)
        self.slack = float(slack)
        self.age_weight = float(age_weight)
        self.fifo_bound = bool(fifo_bound)
        # a request's time alone, for the virtual FIFO server: fitted to the
        # FIFO baseline's service times on the Poisson stream (fixed cost +
        # max(step latency, throughput) over its steps; median ratio 1.00,
        # 10th / 90th percentile 0.86 / 1.17)
        self.est_overhead_us = float(est_overhead_us)
        self.est_step_us = float(est_step_us)
        self.est_traj_step_us = float(est_traj_step_us)
        self._vfifo = 0.0  # virtual FIFO server: completion of the last request
        self._urgent = None  # the request pick() runs alone to its end
        if self.window_ms is not None and (self.window_ms <= 0 or self.step_us <= 0):
            raise ValueError("window_ms and step_us must be positive")
        self.clock = clock
        self.failed = []
        self.timed_out = []
        self.cancelled = []
        self.peak_bytes = 0
        self.peak_active = 0
        self.n_groups = int(getattr(executor, "n_groups", 1))
        self._events = [deque() for _ in range(self.n_groups)]
        self.retiring = []
        self.waiting = deque()
        self.active = []
        self.finishing = []
        self.completed = []
        self.rejected = []

    # ------------------------------------------------------------ requests
    def submit(self, tag, problem, n_traj, seed, arrival=None, timeout=None):
        """Queue a request; `timeout` (seconds after arrival) drops it if it
        has not finished by then."""
        arrival = self.clock() if arrival is None else arrival
        req = Request(tag, problem, n_traj, seed, arrival,
                      None if timeout is None else arrival + timeout)
        req.bytes = self.x.footprint(problem, n_traj)
        req.n_steps = self.x.steps(problem)
        if req.bytes > self.alloc.size:
            req.state = "rejected"
            self.rejected.append(req)
            return req
        # completion on a server that runs the requests one at a time in
        # arrival order, each at its estimated time alone
        req.fifo_finish = max(self._vfifo, arrival) + \
            (self.est_overhead_us + self.est_us(req, req.n_steps + 1)) * 1e-6
        self._vfifo = req.fifo_finish
        self.waiting.append(req)
        return req

    def cancel(self, tag):
        """Drop a waiting request, or stop an admitted one at the next window."""
        for r in list(self.waiting):
            if r.tag == tag:
                self.waiting.remove(r)
                r.state = "cancelled"
                self.cancelled.append(r)
                return True
        for r in self.active:
            if r.tag == tag:
                r.state = "cancelling"
                return True
        return False

    def admit(self):
        """Admit waiting requests in arrival order while memory and table
        slots allow; a request that does not fit yet does not block smaller
        later ones."""
        admitted = []
        now = self.clock()
        for r in list(self.waiting):
            if r.deadline is not None and now > r.deadline:
                self.waiting.remove(r)
                r.state = "timeout"
                self.timed_out.append(r)
                continue
            if not self.free_slots:
                break
            off = self.alloc.alloc(r.bytes)
            if off is None:
                continue
            self.waiting.remove(r)
            r.offset = off
            r.slot = self.free_slots.popleft()
            r.admitted = now
            try:
                self.x.init(r)
            except Exception as e:  # the library refused it: release and report
                r.error = e
                r.state = "failed"
                self._release(r)
                self.failed.append(r)
                continue
            r.state = "active"
            self.active.append(r)
            admitted.append(r)
        self.peak_bytes = max(self.peak_bytes, self.alloc.bytes_used)
        self.peak_active = max(self.peak_active, len(self.active) + len(self.finishing))
        return admitted

    # ---------------------------------------------------------- scheduling
    def remaining(self, r):
        return r.n_traj * (r.n_steps + 1 - r.k_next)

    def pick(self):
        """Requests the next window advances."""
        now = self.clock()
        for r in self.active:
            if r.deadline is not None and now > r.deadline and r.state == "active":
                r.state = "timing_out"
        run = [r for r in self.active if r.state == "active"]
        self._urgent = None
        if self.policy == "ps":
            return run
        if self.policy == "srpt":
            # least estimated time left first, less the waiting time times
            # age_weight (a request that has waited long enough goes first);
            # with fifo_bound, a request that would finish more than one
            # window after its virtual FIFO completion (fifo_finish - now -
            # time left < -window) runs alone to the end of its pulse,
            # earliest fifo_finish first, as it would on the FIFO server
            late = (self.window_ms if self.window_ms is not None else 40.0) * 1e-3

            def key(r):
                if self.fifo_bound:
                    left = self.est_us(r, r.n_steps + 1 - r.k_next) * 1e-6
                    if r.fifo_finish - now - left < -late:
                        return (0, r.fifo_finish)
                return (1, self.time_left_us(r) - self.age_weight * 1e6 * (now - r.arrival))
            keys = {id(r): key(r) for r in run}
            run.sort(key=lambda r: keys[id(r)])
            if run and keys[id(run[0])][0] == 0:
                self._urgent = run[0]
                return run[:1]
        elif self.policy == "backfill":
            # the oldest request always runs; the rest fill by least work left
            head = min(run, key=lambda r: r.arrival) if run else None
            run = ([head] if head else []) + sorted((r for r in run if r is not head),
                                                   key=self.remaining)
        else:  # "deadline": arrival + slack x (estimated time alone), earliest first
            run.sort(key=self.deadline)
        chosen, waves = [], 0
        for r in run:
            if waves >= self.fill_waves:
                break
            chosen.append(r)
            waves += (r.n_traj + 63) // 64
        return chosen

    def time_left_us(self, r):
        """Estimated time of the request's remaining steps alone on the device."""
        steps = r.n_steps + 1 - r.k_next
        return max(steps * self.step_us, r.n_traj * steps * self.traj_step_us)

    def est_us(self, r, steps):
        """Fitted time of `steps` steps of the request alone (virtual FIFO)."""
        return max(steps * self.est_step_us, r.n_traj * steps * self.est_traj_step_us)

    def alone_us(self, r):
        """Estimated time of the request's whole pulse alone on the device."""
        steps = r.n_steps + 1
        return max(steps * self.step_us, r.n_traj * steps * self.traj_step_us)

    def deadline(self, r):
        return r.arrival + self.slack * self.alone_us(r) * 1e-6

    def window_for(self, picked):
        """Window length of the next launch (steps)."""
        waves = sum((r.n_traj + 63) // 64 for r in picked)
        if self.window_ms is None:
            stretch = min(self.max_stretch, max(1, self.device_waves // max(waves, 1)))
            return self.window * stretch
        rest = [r.n_steps + 1 - r.k_next for r in picked]
        if len(picked) == 1 and (len(self.active) == 1 and not self.waiting
                                 or picked[0] is self._urgent):
            return max(1, rest[0])
        traj = sum(r.n_traj for r in picked) / max(self.n_groups, 1)
        step = max(self.step_us, traj * self.traj_step_us)  # one step of the launch
        steps = int(self.window_ms * 1e3 / step)
        return max(1, min(max(self.window, steps), min(rest)))

    def entries_for(self, picked, win):
        """(request, k_from, k_to) of the next launch, in launch order.  Every
        request advances `win` steps, except that, in time-targeted windows, a
        request bound by its wavefronts' step latency (alone it would take
        n x traj_step_us < step_us per step) advances as many steps as fit
        into the launch's expected duration at two wavefronts per SIMD, while
        the work so added stays under a quarter of the launch's.  Otherwise a
        request of few trajectories and a long pulse would advance at the pace
        of the launch's throughput-bound ones.  Requests taking more steps
        come first, so that their longer-running packs start first."""
        ents = [(r, r.k_next, min(r.k_next + win, r.n_steps + 1)) for r in picked]
        if self.window_ms is None or len(ents) < 2:
            return ents
        groups = max(self.n_groups, 1)
        t_step = max(self.step_us, sum(r.n_traj for r in picked) / groups * self.traj_step_us)
        dur = win * t_step
        w_lat = int(dur / (2.0 * self.step_us))
        if w_lat <= win:
            return ents
        budget = 0.25 * dur
        out = []
        for r, a, b in ents:  # in priority order: the first picked gain first
            per_step = r.n_traj / groups * self.traj_step_us
            extra = min(r.n_steps + 1, a + w_lat) - b
            if extra > 0 and r.n_traj * self.traj_step_us < self.step_us \
                    and per_step * extra <= budget:
                budget -= per_step * extra
                b += extra
            out.append((r, a, b))
        out.sort(key=lambda e: e[1] - e[2])  # most steps first (stable)
        return out

    def device_busy(self):
        """True while some pack group has `in_flight` windows outstanding."""
        for evs in self._events:
            while evs and self.x.done(evs[0]):
                evs.popleft()
            if len(evs) >= self.in_flight:
                return True
        return False

    def step(self, block=True):
        """One window over the picked requests, launched for every pack group;
        requests that reach the end of their pulse are finalised.  Returns the
        number of requests run.  With block=False nothing is launched (and 0
        returned) while the device already holds `in_flight` windows, so that
        the caller can take arrivals and finished requests meanwhile."""
        if not block and self.device_busy():
            return 0
        picked = self.pick()
        entries = self.entries_for(picked, self.window_for(picked))
        if entries:
            for g in range(self.n_groups):
                evs = self._events[g]
                while len(evs) >= self.in_flight:
                    self.x.wait(evs.popleft())
                evs.append(self.x.window(entries, g))
        for r, _, k_to in entries:
            r.k_next = k_to
        still = []
        for r in self.active:
            if r.state in ("cancelling", "timing_out"):
                # its memory is released once the work queued for it is done
                r.event = self.x.retire(r)
                if r.state == "cancelling":
                    r.state = "cancelled"
                    self.cancelled.append(r)
                else:
                    r.state = "timeout"
                    self.timed_out.append(r)
                self.retiring.append(r)
                continue
            if r.k_next > r.n_steps:
                r.event = self.x.finalize(r)
                r.state = "finishing"
                self.finishing.append(r)
            else:
                still.append(r)
        self.active = still
        return len(entries)

    def poll(self):
        """Collect finished requests and release retired ones; returns the
        finished requests."""
        for r in list(self.retiring):
            if self.x.done(r.event):
                self.retiring.remove(r)
                self._release(r)
        done = []
        for r in list(self.finishing):
            if self.x.done(r.event):
                r.result = self.x.result(r)
                r.finished = self.clock()
                r.state = "done"
                self.finishing.remove(r)
                self._release(r)
                self.completed.append(r)
                done.append(r)
        return done

    def _release(self, r):
        self.alloc.free(r.offset)
        self.free_slots.append(r.slot)

    @property
    def busy(self):
        return bool(self.waiting or self.active or self.finishing or self.retiring)

    def drain(self):
        while self.busy:
            self.admit()
            if self.active:
                self.step()
            self.poll()


def serve_stream(server, stream, t_limit=None, sleep=time.sleep, poll_s=2e-4):
    """Replay a request stream [(arrival_s, problem, n_traj, seed)] in real
    time through the server.  The host never blocks on the device: while the
    device holds its windows it takes arrivals and collects finished
    requests, polling every `poll_s`.  Returns the completed requests."""
    t0 = server.clock()
    pending = deque(sorted(enumerate(stream), key=lambda x: x[1][0]))
    while pending or server.busy:
        now = server.clock() - t0
        if t_limit is not None and now > t_limit:
            break
        while pending and pending[0][1][0] <= now:
            i, (arr, prob, n, seed) = pending.popleft()
            server.submit(i, prob, n, seed, arrival=t0 + arr)
        server.admit()
        launched = server.step(block=False) if server.active else 0
        finished = server.poll()
        if launched or finished:
            continue
        # nothing to do before the next arrival, window end or result
        gap = pending[0][1][0] - (server.clock() - t0) if pending else poll_s
        if server.active or server.finishing or server.retiring:
            gap = min(gap, poll_s)
        sleep(max(0.0, min(gap, 0.01)))
    return server.completed


def fifo_stream(stream, run_one, clock=time.perf_counter, sleep=time.sleep):
    """Baseline server: requests one at a time, in arrival order, each run to
    completion by `run_one(problem, n_traj, seed)` before the next starts."""
    t0 = clock()
    done = []
    for i, (arr, prob, n, seed) in sorted(enumerate(stream), key=lambda x: x[1][0]):
        wait = arr - (clock() - t0)
        if wait > 0:
            sleep(wait)
        r = Request(i, prob, n, seed, t0 + arr)
        r.admitted = clock()
        r.result = run_one(prob, n, seed)
        r.finished = clock()
        r.state = "done"
        done.append(r)
    return done


def plain_fp64_runner(h_max, h_step, stream=None):
    """run_one for fifo_stream: the whole FP64 path of one request (sampling,
    propagation, dipole, spectrum), synchronised at its end."""
    import torch
    from . import run

    def run_one(prob, n, seed):
        out = run([prob], [n], [seed], precision="fp64", h_max=h_max, h_step=h_step,
                  stream=stream)
        torch.cuda.synchronize()
        return {"v": out["v"][0].cpu(), "yield": out["yield"][0].cpu()}

    return run_one


def latency_stats(reqs):
    lat = sorted(r.finished - r.arrival for r in reqs)
    if not lat:
        return {}
    pick = lambda q: lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)]
    return {"n": len(lat), "p50_s": pick(0.50), "p99_s": pick(0.99), "mean_s": sum(lat) / len(lat),
            "max_s": lat[-1]}

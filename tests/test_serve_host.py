"""Host logic of the serving loop (allocator, admission, scheduling, cancel,
timeout, refused admission) driven by a host-only executor, plus the serving
entry points' argument checks, which return before any device call."""
import ctypes as C
import random

import pytest

from paper_2608_13686_amd import _abi
from paper_2608_13686_amd.serve import (PoolAllocator, Server, fifo_stream, latency_stats,
                                        serve_stream)
import workloads as W


# ------------------------------------------------------------------ allocator
def test_allocator_random_against_interval_model():
    rng = random.Random(7)
    size = 1 << 20
    A = PoolAllocator(size)
    live = {}
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off = rng.choice(list(live))
            A.free(off)
            del live[off]
        else:
            n = rng.randint(1, 40000)
            off = A.alloc(n)
            if off is None:
                # refused only when no free range is large enough
                assert A.largest_free() < (n + 255) // 256 * 256
                continue
            assert off % 256 == 0 and off + n <= size
            for o, m in live.items():
                assert off + n <= o or o + m <= off, "overlapping ranges"
            live[off] = n
        assert A.bytes_used + sum(l for _, l in A.free_list) == size
    for off in list(live):
        A.free(off)
    assert A.free_list == [(0, size)] and A.bytes_used == 0


def test_allocator_coalesces_neighbours():
    A = PoolAllocator(4096)
    a, b, c = A.alloc(1000), A.alloc(1000), A.alloc(1000)
    assert (a, b, c) == (0, 1024, 2048)
    A.free(a)
    A.free(c)
    assert A.free_list == [(0, 1024), (2048, 2048)]  # c merged with the tail
    assert A.alloc(2049) is None  # 2304 bytes after alignment: no hole is large enough
    A.free(b)
    assert A.free_list == [(0, 4096)]
    assert A.alloc(4096) == 0


# -------------------------------------------------------------- fake executor
class FakeExec:
    """Host-only executor with two pack groups: records every call and checks
    that concurrently admitted requests never share memory or a table slot."""

    n_groups = 2

    def __init__(self, fail_tags=()):
        self.windows = {}
        self.finalized = []
        self.retired = []
        self.launches = []
        self.live = {}
        self.fail_tags = set(fail_tags)
        self.waits = 0

    def footprint(self, problem, n):
        return 4096 + 128 * n

    def steps(self, problem):
        return problem["N"]

    def init(self, r):
        if r.tag in self.fail_tags:
            raise _abi.SfhkError(2, "injected ENOMEM")
        for t, (off, nb, slot) in self.live.items():
            assert slot != r.slot
            assert r.offset + r.bytes <= off or off + nb <= r.offset
        self.live[r.tag] = (r.offset, r.bytes, r.slot)
        self.windows[r.tag] = {g: [] for g in range(self.n_groups)}

    def window(self, entries, group=0):
        assert entries and 0 <= group < self.n_groups
        self.launches.append((group, [(r.tag, a, b) for r, a, b in entries]))
        for r, a, b in entries:
            assert r.tag in self.live
            self.windows[r.tag][group].append((a, b))
        return len(self.launches)

    def finalize(self, r):
        self.finalized.append(r.tag)
        self.live.pop(r.tag)
        return 0

    def retire(self, r):
        self.retired.append(r.tag)
        self.live.pop(r.tag)
        return 0

    def done(self, ev):
        return True

    def wait(self, ev):
        self.waits += 1

    def result(self, r):
        w = self.windows[r.tag]
        assert all(w[g] == w[0] for g in w), "pack groups advanced differently"
        return {"windows": list(w[0])}


def _prob(N):
    return {"N": N}


def test_server_windows_cover_each_request_once():
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 22, max_requests=4, window=100, in_flight=2, max_stretch=1,
               window_ms=None, policy="ps")
    sizes = [(250, 1000), (99, 64), (1000, 3000), (100, 5), (0, 10), (333, 7000)]
    for i, (N, n) in enumerate(sizes):
        S.submit(i, _prob(N), n, seed=i)
    S.drain()
    assert sorted(r.tag for r in S.completed) == list(range(len(sizes)))
    for r in S.completed:
        w = r.result["windows"]
        assert w[0][0] == 0 and w[-1][1] == r.n_steps + 1
        assert all(a < b and b - a <= 100 for a, b in w)
        assert all(w[i][1] == w[i + 1][0] for i in range(len(w) - 1))
    assert sorted(x.finalized) == list(range(len(sizes)))
    assert S.peak_active <= 4 and not x.live
    assert S.alloc.free_list == [(0, 1 << 22)]
    # at most in_flight launches per pack group are ever outstanding
    assert x.waits >= len(x.launches) - 2 * x.n_groups


def test_admission_never_exceeds_pool_and_slots():
    x = FakeExec()
    pool = 600_000
    S = Server(x, pool_bytes=pool, max_requests=3, window=64, window_ms=None)
    rng = random.Random(3)
    tags = 0
    for _ in range(40):
        for _ in range(rng.randint(0, 3)):
            S.submit(tags, _prob(rng.randint(10, 400)), rng.randint(1, 4000), seed=tags)
            tags += 1
        S.admit()
        assert S.alloc.bytes_used <= pool
        assert len(S.active) + len(S.finishing) <= 3
        if S.active:
            S.step()
        S.poll()
    S.drain()
    assert len(S.completed) + len(S.rejected) == tags
    assert S.peak_bytes <= pool


def test_big_request_waits_small_ones_pass_and_oversized_is_rejected():
    x = FakeExec()
    fp = x.footprint(None, 1000)
    S = Server(x, pool_bytes=2 * fp, max_requests=8, window=50, window_ms=None)
    S.submit("a", _prob(500), 1000, 0)
    S.admit()
    S.submit("big", _prob(100), 1500, 1)  # needs more than what is left
    S.submit("small", _prob(100), 10, 2)
    S.submit("huge", _prob(100), 10**6, 3)  # larger than the whole pool
    adm = S.admit()
    assert [r.tag for r in adm] == ["small"]
    assert [r.tag for r in S.rejected] == ["huge"]
    S.drain()
    assert {r.tag for r in S.completed} == {"a", "big", "small"}


def test_cancel_waiting_and_active():
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 22, max_requests=1, window=10, window_ms=None)
    S.submit("run", _prob(100), 100, 0)
    S.submit("wait", _prob(100), 100, 1)
    S.admit()
    S.step()
    assert S.cancel("wait") and S.cancel("run")
    assert not S.cancel("nobody")
    S.step()
    S.drain()
    assert {r.tag for r in S.cancelled} == {"run", "wait"}
    assert not S.completed and not x.finalized and x.retired == ["run"]
    assert S.alloc.bytes_used == 0 and len(S.free_slots) == 1


def test_timeout_waiting_and_active():
    t = [0.0]
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 22, max_requests=1, window=10, clock=lambda: t[0],
               window_ms=None)
    S.submit("a", _prob(1000), 100, 0, timeout=5.0)
    S.submit("b", _prob(10), 100, 1, timeout=1.0)
    S.admit()
    S.step()
    t[0] = 2.0
    S.admit()  # b never got a slot before its deadline
    t[0] = 6.0
    S.step()  # a passes its deadline while running
    S.drain()
    assert {r.tag for r in S.timed_out} == {"a", "b"}
    assert S.alloc.bytes_used == 0 and len(S.free_slots) == 1


def test_refused_admission_releases_memory():
    x = FakeExec(fail_tags={"bad"})
    S = Server(x, pool_bytes=1 << 22, max_requests=2, window=100, window_ms=None)
    S.submit("bad", _prob(100), 10, 0)
    S.submit("good", _prob(100), 10, 1)
    S.drain()
    assert [r.tag for r in S.failed] == ["bad"] and isinstance(S.failed[0].error, _abi.SfhkError)
    assert [r.tag for r in S.completed] == ["good"]
    assert S.alloc.bytes_used == 0


def test_srpt_picks_least_remaining_work_and_fills():
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 30, max_requests=8, window=100, policy="srpt",
               fill_waves=20, window_ms=None)
    S.submit("long", _prob(10_000), 640, 0)   # 10 waves, much work
    S.submit("short", _prob(100), 640, 1)     # 10 waves, little work
    S.submit("mid", _prob(1000), 640, 2)
    S.admit()
    S.step()
    assert [t for t, _, _ in x.launches[0][1]] == ["short", "mid"]
    assert x.launches[1][0] == 1 and x.launches[1][1] == x.launches[0][1]
    S.drain()
    assert [r.tag for r in S.completed][:2] == ["short", "mid"]


def test_srpt_default_fill_is_four_devices():
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 30, max_requests=8, window=100, device_waves=16,
               window_ms=None)
    assert S.policy == "srpt" and S.fill_waves == 64
    S.submit("a", _prob(100), 1920, 0)   # 30 waves
    S.submit("b", _prob(200), 2560, 1)   # 40 waves: reaches the fill
    S.submit("c", _prob(300), 6400, 2)  # most work: waits
    S.admit()
    S.step()
    assert [t for t, _, _ in x.launches[0][1]] == ["a", "b"]


def test_backfill_runs_the_oldest_and_deadline_orders_by_slack():
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 30, max_requests=8, window=100, policy="backfill",
               fill_waves=20, window_ms=None)
    S.submit("old_long", _prob(10_000), 640, 0, arrival=0.0)
    S.submit("short", _prob(100), 640, 1, arrival=1.0)
    S.submit("mid", _prob(1000), 640, 2, arrival=2.0)
    S.admit()
    S.step()
    assert [t for t, _, _ in x.launches[0][1]] == ["old_long", "short"]
    # deadline = arrival + slack x max(steps x step_us, n x steps x traj_step_us)
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 30, max_requests=8, window=100, policy="deadline",
               fill_waves=1, window_ms=None, step_us=1.0, traj_step_us=0.0, slack=2.0)
    S.submit("a", _prob(999_999), 64, 0, arrival=0.0)   # deadline 0 + 2 x 1.0 s
    S.submit("b", _prob(99_999), 64, 1, arrival=1.9)    # deadline 1.9 + 2 x 0.1 s > 2.0
    S.admit()
    S.step()
    assert [t for t, _, _ in x.launches[0][1]] == ["a"]
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 30, max_requests=8, window=100, policy="deadline",
               fill_waves=1, window_ms=None, step_us=1.0, traj_step_us=0.0, slack=2.0)
    S.submit("a", _prob(999_999), 64, 0, arrival=0.0)
    S.submit("b", _prob(99_999), 64, 1, arrival=1.0)    # deadline 1.2 < 2.0
    S.admit()
    S.step()
    assert [t for t, _, _ in x.launches[0][1]] == ["b"]


def test_non_blocking_step_waits_for_a_free_window():
    class SlowExec(FakeExec):
        n_groups = 1

        def __init__(self):
            super().__init__()
            self.finished = set()

        def done(self, ev):
            return ev in self.finished

    x = SlowExec()
    S = Server(x, pool_bytes=1 << 22, max_requests=4, window=10, in_flight=2, window_ms=None,
               max_stretch=1)
    S.submit("r", _prob(100), 64, 0)  # 11 windows of 10 steps
    S.admit()
    assert S.step(block=False) == 1 and S.step(block=False) == 1
    assert S.device_busy()
    assert S.step(block=False) == 0 and len(x.launches) == 2 and x.waits == 0
    x.finished.add(1)  # the first window ends
    assert not S.device_busy()
    assert S.step(block=False) == 1 and len(x.launches) == 3
    assert S.step(block=False) == 0
    x.finished.update(range(0, 100))  # every later window (and the finalize, 0) ends at once
    while S.busy:
        S.step(block=False)
        S.poll()
    assert [r.tag for r in S.completed] == ["r"] and x.waits == 0


def test_serve_stream_and_fifo_with_fake_clock():
    t = [0.0]

    def sleep(dt):
        t[0] += max(dt, 1e-4)

    def clock():
        t[0] += 1e-4  # every host action costs a little time
        return t[0]

    stream = [(0.01 * i, _prob(50 + 10 * i), 100 + i, i) for i in range(12)]
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 22, max_requests=4, window=32, clock=clock, window_ms=None)
    done = serve_stream(S, stream, sleep=sleep)
    assert sorted(r.tag for r in done) == list(range(12))
    st = latency_stats(done)
    assert st["n"] == 12 and 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"]
    assert all(r.finished >= r.arrival for r in done)
    t[0] = 0.0
    fifo = fifo_stream(stream, lambda p, n, s: {"n": n}, clock=clock, sleep=sleep)
    assert [r.tag for r in fifo] == list(range(12))
    assert all(r.finished >= r.arrival for r in fifo)


def test_small_launches_stretch_their_window():
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 26, max_requests=4, window=100, device_waves=64,
               max_stretch=8, window_ms=None, policy="ps")
    S.submit("small", _prob(5000), 64 * 10, 0)   # 10 waves: window x 6
    S.admit()
    S.step()
    assert x.launches[0][1] == [("small", 0, 600)]
    S.submit("big", _prob(5000), 64 * 100, 1)    # with it, 110 waves: no stretch
    S.admit()
    S.step()
    assert x.launches[-1][1] == [("small", 600, 700), ("big", 0, 100)]
    S.drain()
    w = S.completed[0].result["windows"]
    assert w[-1][1] == 5001 and all(w[i][1] == w[i + 1][0] for i in range(len(w) - 1))


def test_time_targeted_windows():
    """A lone request runs to the end of its pulse in one window; with others
    active a window lasts about window_ms (one step of a launch of n
    trajectories: max(step_us, n traj_step_us)), at least `window` steps, and
    ends with the shortest picked request."""
    x = FakeExec()
    x.n_groups = 1
    S = Server(x, pool_bytes=1 << 30, max_requests=8, window=50, device_waves=64,
               window_ms=1.0, step_us=2.0, traj_step_us=1e-3)
    S.submit("alone", _prob(5000), 64 * 10, 0)
    S.admit()
    S.step()
    assert x.launches[0][1] == [("alone", 0, 5001)]
    S.drain()
    x = FakeExec()
    x.n_groups = 1
    S = Server(x, pool_bytes=1 << 30, max_requests=8, window=50, device_waves=64,
               window_ms=1.0, step_us=2.0, traj_step_us=1e-3)
    S.submit("a", _prob(5000), 64 * 40, 0)    # 2560 trajectories
    S.submit("b", _prob(9000), 64 * 40, 1)    # 5120 in all: 5.12 us per step -> 195 steps
    S.admit()
    S.step()
    assert x.launches[0][1] == [("a", 0, 195), ("b", 0, 195)]
    S.submit("c", _prob(100), 64, 2)          # shortest: the window ends with it
    S.admit()
    S.step()
    assert x.launches[1][1] == [("c", 0, 101), ("a", 195, 296), ("b", 195, 296)]
    S.drain()
    for r in S.completed:
        w = r.result["windows"]
        assert w[0][0] == 0 and w[-1][1] == r.n_steps + 1
        assert all(w[i][1] == w[i + 1][0] for i in range(len(w) - 1))
    # every launch is at least `window` steps unless one of its requests ends
    ends = {r.tag: r.n_steps + 1 for r in S.completed}
    for _, ent in x.launches:
        assert all(b - a == ent[0][2] - ent[0][1] for _, a, b in ent)
        assert ent[0][2] - ent[0][1] >= 50 or any(b == ends[t] for t, _, b in ent)


def test_latency_bound_request_takes_more_steps():
    """Beside a throughput-bound request, a request of few trajectories
    (alone bound by its step latency) advances as many steps as fit into the
    launch's expected duration at two wavefronts per SIMD, and comes first in
    the launch; its windows still cover its pulse once."""
    x = FakeExec()
    x.n_groups = 1
    S = Server(x, pool_bytes=1 << 30, max_requests=8, window=50, device_waves=64,
               window_ms=1.0, step_us=2.0, traj_step_us=1e-3)
    S.submit("big", _prob(9000), 64 * 200, 0)  # 12,800 trajectories: 12.8 us per step alone
    S.submit("small", _prob(9000), 64, 1)      # 64: bound by the 2 us step latency
    S.admit()
    S.step()
    # one launch step: 12,864 x 1e-3 = 12.864 us -> 77 steps (~1 ms); at
    # 2 x 2 us per step the small request fits 990.5 / 4 = 247 steps
    assert x.launches[0][1] == [("small", 0, 247), ("big", 0, 77)]
    S.drain()
    for r in S.completed:
        w = r.result["windows"]
        assert w[0][0] == 0 and w[-1][1] == r.n_steps + 1
        assert all(w[i][1] == w[i + 1][0] for i in range(len(w) - 1))
    small = next(r for r in S.completed if r.tag == "small")
    big = next(r for r in S.completed if r.tag == "big")
    assert len(small.result["windows"]) < len(big.result["windows"])


def test_extra_steps_stay_within_a_quarter_of_the_launch():
    """Latency-bound requests gain steps in priority order only while the
    work they add stays under a quarter of the launch's expected duration;
    throughput-bound requests never gain."""
    x = FakeExec()
    x.n_groups = 1
    S = Server(x, pool_bytes=1 << 30, max_requests=8, window=50, device_waves=64,
               window_ms=1.0, step_us=2.0, traj_step_us=1e-3, fifo_bound=False)
    big = S.submit("big", _prob(9000), 64 * 200, 0)
    smalls = [S.submit(f"s{i}", _prob(9000), 64 * 15, 1 + i) for i in range(4)]
    S.admit()
    picked = [smalls[0], smalls[1], smalls[2], smalls[3], big]
    win = S.window_for(picked)
    ents = S.entries_for(picked, win)
    steps = {r.tag: b - a for r, a, b in ents}
    t_step = max(2.0, (64 * 200 + 4 * 64 * 15) * 1e-3)
    dur = win * t_step
    w_lat = int(dur / 4.0)
    per = 64 * 15 * 1e-3 * (w_lat - win)       # added work of one small request (us)
    n_gain = int(0.25 * dur // per)
    assert 0 < n_gain < 4                       # the budget binds part-way
    assert [steps[f"s{i}"] for i in range(4)] == [w_lat] * n_gain + [win] * (4 - n_gain)
    assert steps["big"] == win
    # launch order: the requests with more steps first, the rest as picked
    assert [r.tag for r, _, _ in ents] == [f"s{i}" for i in range(n_gain)] + \
        [f"s{i}" for i in range(n_gain, 4)] + ["big"]


def test_srpt_bounds_lateness_against_fifo():
    """A request more than one window behind its completion on a virtual FIFO
    server (one request at a time in arrival order, each at its estimated
    time alone) runs alone; until then shorter requests overtake it."""
    now = [0.0]
    x = FakeExec()
    S = Server(x, pool_bytes=1 << 30, max_requests=8, device_waves=64, window_ms=40.0,
               step_us=4.0, traj_step_us=1e-5, est_overhead_us=0.0, est_step_us=4.0,
               est_traj_step_us=1e-5, clock=lambda: now[0])
    big = S.submit("big", _prob(20_000), 64 * 100, 0, arrival=0.0)    # 80 ms alone
    small = S.submit("small", _prob(1_000), 64, 1, arrival=0.0)       # 4 ms alone
    assert abs(big.fifo_finish - 0.080004) < 1e-9
    assert abs(small.fifo_finish - (big.fifo_finish + 0.004004)) < 1e-9
    S.admit()
    assert [r.tag for r in S.pick()] == ["small", "big"]
    now[0] = 0.03   # big 30 ms late: within one window
    assert [r.tag for r in S.pick()] == ["small", "big"]
    now[0] = 0.05   # 50 ms late: alone, to the end of its pulse
    assert [r.tag for r in S.pick()] == ["big"]
    S.step()
    assert x.launches[-1][1] == [("big", 0, 20_001)]
    S2 = Server(FakeExec(), pool_bytes=1 << 30, max_requests=8, device_waves=64,
                window_ms=40.0, step_us=4.0, traj_step_us=1e-5, fifo_bound=False,
                clock=lambda: now[0])
    S2.submit("big", _prob(20_000), 64 * 100, 0, arrival=0.0)
    S2.submit("small", _prob(1_000), 64, 1, arrival=0.0)
    S2.admit()
    assert [r.tag for r in S2.pick()] == ["small", "big"]


def test_server_rejects_bad_config():
    with pytest.raises(ValueError):
        Server(FakeExec(), 1 << 20, policy="lifo", window_ms=None)
    with pytest.raises(ValueError):
        Server(FakeExec(), 1 << 20, window=0, window_ms=None)
    with pytest.raises(ValueError):
        Server(FakeExec(), 1 << 20, window_ms=-1.0)


# -------------------------------------------------- C ABI (host-side checks)
def _h2():
    return _abi.make_problems([W.h2_softcore(0.0)])


def test_request_footprint_and_layout():
    L = _abi.lib()
    p = _h2()
    nb = L.sfhk_request_bytes(p, 4096, 801)
    nb2 = L.sfhk_request_bytes(p, 8192, 801)
    assert 0 < nb < nb2
    # state (47 doubles) + initial conditions and packing (> 90 B) per trajectory
    assert nb2 - nb >= 4096 * (47 * 8 + 90)
    offs = (C.c_size_t * 4)()
    assert L.sfhk_request_layout(p, 4096, 801, offs) == 0
    o = list(offs)
    assert all(x % 256 == 0 for x in o) and o == sorted(o) and o[3] + 801 * 8 <= nb
    assert L.sfhk_request_table_bytes(0) == 0
    assert L.sfhk_request_table_bytes(7) == 7 * L.sfhk_request_table_bytes(1) > 0
    assert L.sfhk_request_bytes(p, 10, -1) == 0


def test_request_entry_points_reject_bad_arguments():
    L = _abi.lib()
    p = _h2()
    nb = L.sfhk_request_bytes(p, 1000, 10)
    fake = C.c_void_p(0x10000)  # never dereferenced: every call below fails its checks first
    E_INVALID, E_NOMEM = 1, 2
    assert L.sfhk_request_init(p, 1000, 1, 0, 0.1, 10, fake, nb - 1, fake, 4, 0, None) == E_NOMEM
    assert L.sfhk_request_init(p, 1000, 1, 0, 0.1, 10, fake, nb, fake, 4, 4, None) == E_INVALID
    assert L.sfhk_request_init(p, 1000, 1, 0, 0.1, 10, None, nb, fake, 4, 0, None) == E_INVALID
    assert L.sfhk_request_init(p, 0, 1, 0, 0.1, 10, fake, nb, fake, 4, 0, None) == E_INVALID
    assert L.sfhk_request_init(p, 1000, 1, 0, -0.1, 10, fake, nb, fake, 4, 0, None) == E_INVALID
    one = (C.c_int32 * 1)
    n64 = (C.c_uint64 * 1)(1000)
    win = L.sfhk_serve_window
    assert win(fake, 4, 1, one(4), n64, one(0), one(10), 0, 1, None) == E_INVALID
    assert win(fake, 4, 1, one(0), n64, one(10), one(10), 0, 1, None) == E_INVALID
    assert win(fake, 4, 1, one(0), n64, one(-1), one(10), 0, 1, None) == E_INVALID
    assert win(fake, 4, 1, one(0), n64, one(0), one(10), 2, 2, None) == E_INVALID  # group >= n
    assert win(fake, 4, 1, one(0), n64, one(0), one(10), 0, 0, None) == E_INVALID
    assert win(fake, 4, 1, one(0), n64, one(0), one(10), 0, 65, None) == E_INVALID
    assert win(None, 4, 0, None, None, None, None, 0, 1, None) == E_INVALID
    assert win(fake, 4, 0, None, None, None, None, 0, 1, None) == 0  # nothing to do
    big = (C.c_uint64 * 1)(1 << 40)
    assert win(fake, 4, 1, one(0), big, one(0), one(10), 0, 1, None) == 5
    assert L.sfhk_request_finalize(p, 10, fake, 4, 4, None) == E_INVALID
    assert L.sfhk_request_finalize(p, -1, fake, 4, 0, None) == E_INVALID

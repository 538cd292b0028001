"""Serving scheduler on the CPU with a simulated executor and a manual
clock: budget admission, FIFO order, continuous batching, starvation
freedom, launch failures, the watchdog and rejection of oversize requests."""
import math

import pytest

from paper_2203_10587_amd.serve import Executor, Server, poisson_trace


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor(Executor):
    def __init__(self, clock, caps=(8, 4), slot_bytes=(100, 1000), cost=(0.001, 0.01),
                 fail_calls=(), hang_calls=()):
        self.clock = clock
        self.caps, self.sb, self.cost = caps, slot_bytes, cost
        self.calls = []
        self.fail_calls, self.hang_calls = set(fail_calls), set(hang_calls)
        self.busy = {}

    def grids(self):
        return list(range(len(self.caps)))

    def capacity(self, g):
        return self.caps[g]

    def slot_bytes(self, g):
        return self.sb[g]

    def launch(self, g, first, seeds):
        idx = len(self.calls)
        self.calls.append((self.clock(), g, first, list(seeds)))
        if idx in self.fail_calls:
            raise RuntimeError("injected launch failure")
        # one device stream per grid: windows of a grid run back to back
        start = max(self.clock(), self.busy.get(g, 0.0))
        end = start + self.cost[g] * (1 + 0.1 * len(seeds))
        self.busy[g] = end
        # an injected hang is a completion that never arrives
        return math.inf if idx in self.hang_calls else end

    def done(self, h):
        return self.clock() >= h


def drive(server, clock, dt=1e-4, limit=10.0):
    while not server.idle() and clock.t < limit:
        server.step()
        clock.t += dt


def test_all_done_and_budget_respected():
    clk = Clock()
    ex = FakeExecutor(clk)
    s = Server(ex, budget_bytes=2500, max_window=3, clock=clk)
    for i in range(60):
        s.submit(i % 2, i)
    drive(s, clk)
    st = s.stats(clk.t)
    assert st["done"] == 60 and st["failed"] == 0
    assert s.peak_bytes <= 2500
    assert s.bytes_in_flight == 0


def test_fifo_within_grid_and_slots_in_range():
    clk = Clock()
    ex = FakeExecutor(clk)
    s = Server(ex, max_window=2, clock=clk)
    reqs = [s.submit(0, i) for i in range(20)]
    drive(s, clk)
    launches = [r.t_launch for r in reqs]
    assert launches == sorted(launches)
    assert all(0 <= r.slot < ex.caps[0] for r in reqs)
    # a slot is never used by two windows at once
    live = {}
    for t, g, first, seeds in ex.calls:
        for k in range(first, first + len(seeds)):
            assert k < ex.caps[g]


def test_continuous_batching_joins_while_busy():
    """Requests that arrive while a window runs are launched before that
    window completes, as long as slots and budget allow."""
    clk = Clock()
    ex = FakeExecutor(clk, caps=(8,), slot_bytes=(10,), cost=(0.05,))
    s = Server(ex, max_window=8, clock=clk)
    a = [s.submit(0, i) for i in range(3)]
    s.step()
    assert all(r.status == "running" for r in a)
    clk.t += 0.01
    b = [s.submit(0, 100 + i) for i in range(3)]
    s.step()
    assert all(r.status == "running" for r in b)
    assert all(r.status == "running" for r in a)  # first window still in flight
    drive(s, clk)
    assert all(r.status == "done" for r in a + b)
    assert b[0].t_done > a[0].t_done  # same-grid windows run back to back


def test_budget_serializes_windows():
    clk = Clock()
    ex = FakeExecutor(clk, caps=(8,), slot_bytes=(100,), cost=(0.01,))
    s = Server(ex, budget_bytes=300, max_window=8, clock=clk)
    r = [s.submit(0, i) for i in range(6)]
    s.step()
    assert [x.status for x in r].count("running") == 3
    drive(s, clk)
    assert all(x.status == "done" for x in r)
    assert s.peak_bytes == 300


def test_oversize_request_rejected():
    clk = Clock()
    ex = FakeExecutor(clk)
    s = Server(ex, budget_bytes=500, clock=clk)
    big = s.submit(1, 0)
    small = s.submit(0, 1)
    drive(s, clk)
    assert big.status == "rejected" and "budget" in big.error
    assert small.status == "done"


def test_launch_failure_fails_only_its_window():
    clk = Clock()
    ex = FakeExecutor(clk, fail_calls={0})
    s = Server(ex, max_window=2, clock=clk)
    r = [s.submit(0, i) for i in range(4)]
    drive(s, clk)
    assert [x.status for x in r] == ["failed", "failed", "done", "done"]
    assert "injected" in r[0].error


def test_watchdog_times_out_a_stuck_window():
    clk = Clock()
    ex = FakeExecutor(clk, caps=(4, 4), hang_calls={0})
    s = Server(ex, max_window=2, timeout_s=0.5, clock=clk)
    stuck = [s.submit(0, i) for i in range(2)]
    other = [s.submit(1, 10 + i) for i in range(2)]
    for _ in range(2000):
        s.step()
        clk.t += 1e-3
    assert all(r.status == "failed" and r.error == "timeout" for r in stuck)
    assert all(r.status == "done" for r in other)
    # the stuck slots stay reserved; the rest of the pool keeps serving
    more = [s.submit(0, 20 + i) for i in range(2)]
    for _ in range(200):
        s.step()
        clk.t += 1e-3
    assert all(r.status == "done" for r in more)
    assert all(r.slot >= 2 for r in more)


def test_no_starvation_under_small_flood():
    clk = Clock()
    ex = FakeExecutor(clk, caps=(16, 2), slot_bytes=(10, 500), cost=(0.001, 0.02))
    s = Server(ex, budget_bytes=600, max_window=16, clock=clk)
    big = [s.submit(1, i) for i in range(3)]
    for k in range(400):
        s.submit(0, 1000 + k)
        s.step()
        clk.t += 5e-4
    drive(s, clk)
    assert all(r.status == "done" for r in big)


def test_poisson_trace_shape():
    tr = poisson_trace(2000.0, 2.0, 4, seed=1)
    assert 3600 < len(tr) < 4400
    ts = [t for t, _, _ in tr]
    assert ts == sorted(ts) and 0 <= ts[0] and ts[-1] <= 2.0
    assert {g for _, g, _ in tr} == {0, 1, 2, 3}
    assert tr == poisson_trace(2000.0, 2.0, 4, seed=1)


class InputExecutor(FakeExecutor):
    """A fake that takes caller iterates (x of n = 3, lam of m = 2 entries)
    and 'evaluates' f = sum(x) * sigma into a slot store."""

    def __init__(self, clock, **kw):
        super().__init__(clock, **kw)
        self.inputs_seen = []
        self.slots = {}

    def check_inputs(self, g, x, lam):
        if len(x) != 3 or len(lam) != 2:
            raise ValueError("x takes 3 and lam 2 entries")

    def launch(self, g, first, seeds, inputs=None):
        self.inputs_seen.append((first, inputs))
        for i, s in enumerate(seeds):
            inp = inputs[i] if inputs else None
            self.slots[(g, first + i)] = (sum(inp[0]) * inp[2]) if inp else float(s)
        return super().launch(g, first, seeds)

    copy_delay = 0.0

    def collect(self, g, slot):
        return {"f": self.slots[(g, slot)]}

    def mark(self, g):
        # the copies queue behind the grid's work, then take copy_delay
        return max(self.clock(), self.busy.get(g, 0.0)) + self.copy_delay


def test_caller_iterates_and_results():
    """Requests with their own (x, lam, sigma) reach the executor slot by
    slot beside seeded ones; wrong sizes are rejected at submit; with
    keep_results every finished request holds its own outputs."""
    clock = Clock()
    ex = InputExecutor(clock)
    srv = Server(ex, budget_bytes=10_000, clock=clock, keep_results=True)
    a = srv.submit(0, seed=7)
    b = srv.submit(0, x=[1.0, 2.0, 3.0], lam=[0.0, 0.0], sigma=2.0)
    c = srv.submit(0, x=[1.0], lam=[0.0, 0.0])
    d = srv.submit(0, x=[1.0, 1.0, 1.0])
    assert c.status == "rejected" and "inputs" in c.error
    assert d.status == "rejected" and "together" in d.error
    drive(srv, clock)
    assert a.status == b.status == "done"
    assert a.result == {"f": 7.0} and b.result == {"f": 12.0}
    assert b.inputs is None  # released once copied
    first, inputs = ex.inputs_seen[0]
    assert inputs[0] is None and inputs[1][2] == 2.0


def test_seeded_only_executor_rejects_inputs():
    clock = Clock()
    srv = Server(FakeExecutor(clock), clock=clock)
    r = srv.submit(0, x=[1.0], lam=[1.0])
    assert r.status == "rejected"


def test_pool_finds_any_free_slot():
    """A window is placed whenever some slot is free, also when the slot at
    the head and slot 0 are both taken; runs never wrap past the last slot."""
    from paper_2203_10587_amd.serve import _Pool
    p = _Pool(6)
    assert p.alloc(2) == (0, 2) and p.alloc(3) == (2, 3)   # slots 0..4 taken, head 5
    assert p.alloc(4) == (5, 1)                            # the run stops at the end
    assert p.alloc(1) is None                              # all six taken
    p.free(3, 1)                                           # head 0 taken, slot 3 free
    assert p.alloc(2) == (3, 1)
    p.free(0, 2)
    p.free(4, 1)
    assert p.alloc(8) == (4, 1)                            # head was 4; slot 5 taken
    assert p.alloc(8) == (0, 2)
    assert p.alloc(1) is None


def test_kept_results_are_done_only_after_their_copies():
    """With keep_results a finished window's requests wait in 'copying' until
    the executor's mark for the grid completes (the copies have run); only
    then are they 'done', and their slots are free for the next window at
    once (the copies are ordered before it on the grid's stream)."""
    clock = Clock()
    ex = InputExecutor(clock, caps=(2, 2))
    ex.copy_delay = 0.05
    srv = Server(ex, budget_bytes=10_000, clock=clock, keep_results=True)
    a = srv.submit(0, seed=3)
    b = srv.submit(0, seed=4)
    srv.step()
    assert a.status == b.status == "running"
    clock.t = 0.02  # the window has finished on the device
    srv.step()
    assert a.status == b.status == "copying" and a.result == {"f": 3.0}
    assert not srv.idle()
    c = srv.submit(0, seed=5)
    srv.step()
    assert c.status == "running"          # the slots were free again
    clock.t = 0.06
    srv.step()
    assert a.status == "copying"          # copies still running
    clock.t = 0.08
    srv.step()
    assert a.status == b.status == "done"
    assert a.t_done == b.t_done == 0.08
    drive(srv, clock)
    assert c.status == "done" and c.result == {"f": 5.0}
    assert srv.idle()


def test_stats_break_latency_into_parts():
    """queue + launch + complete = latency for every request; the parts and
    the peak of windows in flight are reported."""
    clk = Clock()
    ex = FakeExecutor(clk)
    s = Server(ex, max_window=3, clock=clk)
    for i in range(30):
        s.submit(i % 2, i)
    drive(s, clk)
    for r in s.requests:
        parts = (r.t_launch - r.t_arrive) + (r.t_issued - r.t_launch) + (r.t_done - r.t_issued)
        assert abs(parts - r.latency) < 1e-12
    st = s.stats(clk.t)
    assert set(st["parts"]) == {"queue", "launch", "complete"}
    assert st["peak_windows_in_flight"] >= 2  # both grids' windows run together
    assert st["mean_window"] > 1.0            # a burst is taken in windows of several


def test_run_trace_reports_stalls():
    """A pass of the serving loop that takes longer than the stall threshold
    is reported, with its length; the collector can be switched off for the
    trace and is restored afterwards."""
    import gc
    from paper_2203_10587_amd import serve as SV

    class SlowClock(Clock):
        def __call__(self):
            self.t += 1e-4          # every reading advances the clock a little
            if abs(self.t - 0.01) < 5e-5:
                self.t += 0.004     # one 4 ms gap
            return self.t

    clk = SlowClock()
    ex = FakeExecutor(clk)
    s = Server(ex, clock=clk)
    tr = [(0.002 * k, k % 2, k) for k in range(20)]
    was = gc.isenabled()
    st = s.run_trace(tr, gc_off=True)
    assert gc.isenabled() == was
    assert st["done"] == 20
    assert st["stalls"]["count"] >= 1 and st["stalls"]["max_ms"] >= 4.0
    assert st["stalls"]["gc_off"] is True and st["stalls"]["gc_pauses"] == 0
    assert SV.STALL_S * 1e3 == st["stalls"]["threshold_ms"]


def test_stalls_name_the_part_of_the_pass():
    """A stall inside the launch call is attributed to admitting; one in the
    completion poll to retiring; one between passes to neither."""

    class TickClock(Clock):
        def __call__(self):
            self.t += 1e-5
            return self.t

    for where in ("admit", "retire", "other"):
        clk = TickClock()

        class Slow(FakeExecutor):
            slowed = False

            def launch(self, g, first, seeds):
                if where == "admit" and not Slow.slowed:
                    Slow.slowed = True
                    clk.t += 0.004
                return super().launch(g, first, seeds)

            def done(self, h):
                if where == "retire" and not Slow.slowed and self.calls:
                    Slow.slowed = True
                    clk.t += 0.004
                return super().done(h)

        ex = Slow(clk)
        s = Server(ex, clock=clk)
        tr = [(0.002 * k, k % 2, k) for k in range(20)]
        if where == "other":
            orig = s.submit

            def submit(*a, **k):
                if not getattr(s, "_slowed", False):
                    s._slowed = True
                    clk.t += 0.004
                return orig(*a, **k)
            s.submit = submit
        st = s.run_trace(tr)
        assert st["done"] == 20
        long = [x for x in st["stalls"]["longest"] if x[1] >= 4.0]
        assert long and long[0][2] == where, (where, st["stalls"])
        assert st["stalls"]["where"][where] >= 1


def test_collector_setup_precedes_the_trace_clock(monkeypatch):
    """With gc_off the full collection runs before the trace's clock starts,
    so it is neither a stall nor part of any request's latency."""
    import gc

    class TickClock(Clock):
        def __call__(self):
            self.t += 1e-5
            return self.t

    real = gc.collect

    def run(collect_s):
        clk = TickClock()

        def slow_collect(*a, **k):
            clk.t += collect_s  # the collection's time on the trace's clock
            return real(*a, **k)

        monkeypatch.setattr(gc, "collect", slow_collect)
        s = Server(FakeExecutor(clk), clock=clk)
        st = s.run_trace([(0.0005 * k, k % 2, k) for k in range(20)], gc_off=True)
        monkeypatch.setattr(gc, "collect", real)
        assert st["done"] == 20
        return st, [r.latency for r in s.requests]

    st, slow = run(0.07)
    assert st["stalls"]["count"] == 0, st["stalls"]
    _, fast = run(0.0)
    # (the same up to a clock tick or two; a collection on the trace clock
    # would add its 70 ms to the first requests)
    assert len(slow) == len(fast) and all(abs(a - b) <= 1e-3 for a, b in zip(slow, fast))

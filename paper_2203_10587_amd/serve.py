"""Continuous-batching evaluation server.

Requests name a resident grid and either carry their own iterate (x, lambda,
sigma: a solver's request) or a seed, from which the device draws the
iterate and multipliers (the synthetic served workload).  Each is evaluated
(f, grad f, c, J and H) into a slot of that grid's pool; with keep_results
the finished request holds device copies of its outputs (a future: poll
Request.status; once it reads "done" the copies have completed on the
device, so Request.result can be read on any stream).  The scheduler

  - keeps each grid's network resident on the device and one slot pool per
    grid (the instance slots of one batch handle);
  - admits queued requests oldest-first while slots are free and the HBM
    bytes of all in-flight slots stay within the budget; a request whose slot
    alone exceeds the budget is rejected (ACOPF_EBUDGET semantics);
  - launches every admitted window as soon as it is formed, on the grid's own
    stream, so requests that arrive while others are on the GPU join the next
    window and windows of different grids overlap on the device (continuous
    batching);
  - retires each window when its completion event fires, frees its slots
    and budget, and stamps each request's latency;
  - fails a window whose launch raises, and fails (and quarantines the slots
    of) a window that has not completed within the watchdog timeout.

The device work goes through an Executor; GpuExecutor drives the C ABI
(acopf_batch_draw_iterates + acopf_batch_eval_range), and the CPU tests use
a simulated executor with the same interface.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence


@dataclass
class Request:
    rid: int
    grid: int
    seed: int
    t_arrive: float                 # scheduled arrival (latency runs from here)
    t_submit: float = float("nan")  # when the server took it in
    t_launch: float = float("nan")  # admission: its window's launch call began
    t_issued: float = float("nan")  # the launch call returned
    t_done: float = float("nan")    # completion observed by the server
    slot: int = -1
    status: str = "queued"     # queued | running | copying | done | failed | rejected
    error: str = ""
    inputs: Optional[tuple] = None   # (x, lam, sigma) given by the caller, else drawn
    result: Optional[dict] = None    # device outputs once done (keep_results)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


@dataclass
class _Window:
    grid: int
    first: int
    reqs: List[Request]
    handle: object
    t_launch: float
    nbytes: int


class Executor:
    """Device side of the server (one pool of `capacity[g]` slots per grid)."""

    def grids(self) -> Sequence[int]:
        raise NotImplementedError

    def capacity(self, grid: int) -> int:
        raise NotImplementedError

    def slot_bytes(self, grid: int) -> int:
        raise NotImplementedError

    def launch(self, grid: int, first: int, seeds: Sequence[int], inputs=None):
        """Enqueue draw + evaluation of slots [first, first + len(seeds));
        inputs (if given) holds, per slot, None or the request's own
        (x, lam, sigma)."""
        raise NotImplementedError

    def done(self, handle) -> bool:
        raise NotImplementedError

    def check_inputs(self, grid: int, x, lam) -> None:
        """Raise ValueError unless (x, lam) fit the grid."""
        raise TypeError("this executor evaluates drawn iterates only")

    def collect(self, grid: int, slot: int) -> dict:
        """The outputs of a finished slot, kept apart from the pool: copies
        enqueued behind the grid's work, so a later window cannot overwrite
        the slot first; complete once mark(grid) completes."""
        raise NotImplementedError

    def mark(self, grid: int):
        """A handle (polled with done) that completes once everything
        enqueued so far for `grid`, collect copies included, has finished."""
        raise NotImplementedError


class _Pool:
    """Slot occupancy of one grid.  A window takes the contiguous run of free
    slots (at most the wanted number, not wrapping past the last slot) that
    starts at the first free slot found from the rotating head onwards,
    cyclically; it fails only when every slot is taken.  Slots of a window
    that timed out stay occupied, since the device may still write them."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.occ = [False] * self.capacity
        self.head = 0

    def alloc(self, want: int):
        cap = self.capacity
        if want <= 0 or cap <= 0:
            return None
        for i in range(cap):
            start = (self.head + i) % cap
            if self.occ[start]:
                continue
            run = 0
            while run < want and start + run < cap and not self.occ[start + run]:
                run += 1
            for k in range(start, start + run):
                self.occ[k] = True
            self.head = (start + run) % cap
            return start, run
        return None

    def free(self, first: int, k: int):
        for s in range(first, first + k):
            self.occ[s] = False


STALL_S = 0.5e-3  # a gap between two passes of the serving loop longer than this is a stall


class Server:
    def __init__(self, executor: Executor, budget_bytes: int = 8 << 30, max_window: int = 64,
                 timeout_s: float = 10.0, clock: Callable[[], float] = time.perf_counter,
                 keep_results: bool = False):
        self.ex = executor
        self.keep_results = bool(keep_results)
        self.budget = int(budget_bytes)
        self.max_window = int(max_window)
        self.timeout = float(timeout_s)
        self.clock = clock
        self.pools = {g: _Pool(executor.capacity(g)) for g in executor.grids()}
        self.queues: Dict[int, collections.deque] = {g: collections.deque() for g in self.pools}
        self.inflight: Dict[int, collections.deque] = {g: collections.deque() for g in self.pools}
        self.bytes_in_flight = 0
        self.peak_bytes = 0
        self.requests: List[Request] = []
        self.copying: collections.deque = collections.deque()  # (requests, handle)
        self.windows_launched = 0
        self.peak_windows = 0   # windows in flight at once, at most
        self._rr = 0

    # -- intake ---------------------------------------------------------------
    def submit(self, grid: int, seed: int = 0, t_arrive: Optional[float] = None, x=None,
               lam=None, sigma: float = 1.0) -> Request:
        """Queue one evaluation of `grid`: at the caller's iterate (x, lam,
        sigma) if x is given, else at the iterate drawn from `seed`."""
        now = self.clock()
        r = Request(rid=len(self.requests), grid=grid, seed=int(seed),
                    t_arrive=now if t_arrive is None else float(t_arrive), t_submit=now)
        self.requests.append(r)
        if grid not in self.pools:
            r.status, r.error = "rejected", "unknown grid"
            return r
        if (x is None) != (lam is None):
            r.status, r.error = "rejected", "x and lam go together"
            return r
        if x is not None:
            try:
                self.ex.check_inputs(grid, x, lam)
            except (ValueError, TypeError, AttributeError) as exc:
                r.status, r.error = "rejected", f"inputs: {exc}"
                return r
            r.inputs = (x, lam, float(sigma))
        if self.ex.slot_bytes(grid) > self.budget:
            r.status, r.error = "rejected", "request exceeds the HBM budget"
        else:
            self.queues[grid].append(r)
        return r

    # -- progress -------------------------------------------------------------
    def _retire(self, now: float) -> int:
        n = 0
        # requests whose result copies have completed on the device
        while self.copying and self.ex.done(self.copying[0][1]):
            t = self.clock()
            for r in self.copying.popleft()[0]:
                r.t_done, r.status = t, "done"
            n += 1
        for g, q in self.inflight.items():
            keep = collections.deque()
            for w in q:
                if w.handle is not None and self.ex.done(w.handle):
                    now = self.clock()  # when this completion was seen
                    if w.reqs and w.reqs[0].status == "running":
                        for r in w.reqs:
                            r.inputs = None  # copied into the slot long ago
                        if self.keep_results:
                            # copies enqueued behind the window's work, before
                            # the slots can take a later window; the requests
                            # are done once they have completed
                            for r in w.reqs:
                                r.result = self.ex.collect(g, r.slot)
                                r.status = "copying"
                            self.copying.append((w.reqs, self.ex.mark(g)))
                        else:
                            for r in w.reqs:
                                r.t_done, r.status = now, "done"
                    self.pools[g].free(w.first, len(w.reqs))
                    self.bytes_in_flight -= w.nbytes
                    n += 1
                    continue
                if w.reqs and w.reqs[0].status == "running" and now - w.t_launch > self.timeout:
                    # watchdog: fail the requests now; the slots and their bytes
                    # stay reserved until the device finishes with them
                    for r in w.reqs:
                        r.t_done, r.status, r.error = now, "failed", "timeout"
                    n += 1
                keep.append(w)
            self.inflight[g] = keep
        return n

    def _admit(self, now: float) -> int:
        launched = 0
        grids = list(self.pools)
        for step in range(len(grids)):
            g = grids[(self._rr + step) % len(grids)]
            q, pool = self.queues[g], self.pools[g]
            sb = self.ex.slot_bytes(g)
            while q:
                room = (self.budget - self.bytes_in_flight) // sb
                want = min(len(q), self.max_window, room)
                if want <= 0:
                    break
                got = pool.alloc(want)
                if got is None:
                    break
                first, k = got
                reqs = [q.popleft() for _ in range(k)]
                t_call = self.clock()
                try:
                    seeds = [r.seed for r in reqs]
                    if any(r.inputs is not None for r in reqs):
                        h = self.ex.launch(g, first, seeds, [r.inputs for r in reqs])
                    else:
                        h = self.ex.launch(g, first, seeds)
                except Exception as exc:  # a failed launch fails its window only
                    pool.free(first, k)
                    for r in reqs:
                        r.status, r.error, r.t_done = "failed", f"launch: {exc}", now
                    continue
                t_ret = self.clock()
                for i, r in enumerate(reqs):
                    r.slot, r.status = first + i, "running"
                    r.t_launch, r.t_issued = t_call, t_ret
                self.bytes_in_flight += k * sb
                self.peak_bytes = max(self.peak_bytes, self.bytes_in_flight)
                self.inflight[g].append(_Window(g, first, reqs, h, now, k * sb))
                self.windows_launched += 1
                self.peak_windows = max(self.peak_windows,
                                        sum(len(v) for v in self.inflight.values()))
                launched += 1
        self._rr = (self._rr + 1) % max(1, len(grids))
        return launched

    def step(self) -> int:
        now = self.clock()
        n = self._retire(now)
        t1 = self.clock()
        n += self._admit(now)
        self.last_step_s = (t1 - now, self.clock() - t1)  # retire; admit and launch
        return n

    def idle(self) -> bool:
        return (not any(self.queues.values()) and not any(self.inflight.values())
                and not self.copying)

    # -- open-loop driver -------------------------------------------------------
    def run_trace(self, arrivals: Sequence[tuple], progress: Optional[Callable] = None,
                  time_limit_s: float = 600.0, gc_off: bool = False) -> Dict:
        """arrivals: (t_offset_s, grid, seed) sorted by time; requests enter at
        their scheduled time and latency runs from that time (open loop).
        Records every gap of more than STALL_S between two passes of the loop
        (a stall: nothing is admitted or retired meanwhile), with the part of
        the pass that took most of it (retiring, admitting and launching, or
        neither: the arrivals' bookkeeping or time off the CPU), and every
        pause of Python's garbage collector; with gc_off the collector is
        disabled for the trace."""
        import gc
        # the collector is set up before the trace's clock starts: a full
        # collection here would otherwise hold up the first arrivals
        was_enabled = gc.isenabled()
        if gc_off:
            gc.collect()
            gc.freeze()  # what exists now is never traversed again
            gc.disable()
        t0 = self.clock()
        i = 0
        last_report = t0
        stalls = []      # (start, length, where) of gaps between loop passes, s
        gc_pauses = []   # (start, length) of garbage collections, s
        gc_t = [0.0]

        def on_gc(phase, info):
            if phase == "start":
                gc_t[0] = time.perf_counter()
            else:
                gc_pauses.append((gc_t[0] - t0, time.perf_counter() - gc_t[0]))

        gc.callbacks.append(on_gc)
        try:
            prev = t0
            self.last_step_s = (0.0, 0.0)
            while i < len(arrivals) or not self.idle():
                now = self.clock()
                if now - prev > STALL_S:
                    gap = now - prev
                    rs, ad = self.last_step_s
                    where = "retire" if rs > gap / 2 else ("admit" if ad > gap / 2 else "other")
                    stalls.append((prev - t0, gap, where))
                prev = now
                while i < len(arrivals) and t0 + arrivals[i][0] <= now:
                    t, g, s = arrivals[i]
                    self.submit(g, s, t_arrive=t0 + t)
                    i += 1
                self.step()
                if progress and now - last_report > 5.0:
                    progress(i, len(arrivals))
                    last_report = now
                if now - t0 > time_limit_s:
                    break
        finally:
            gc.callbacks.remove(on_gc)
            if gc_off:
                gc.unfreeze()
                if was_enabled:
                    gc.enable()
        st = self.stats(self.clock() - t0)
        in_gc = sum(any(gs < s0 + sl and s0 < gs + gl for gs, gl in gc_pauses)
                    for s0, sl, _ in stalls)
        st["stalls"] = {"threshold_ms": STALL_S * 1e3, "count": len(stalls),
                        "max_ms": max((sl for _, sl, _ in stalls), default=0.0) * 1e3,
                        "total_ms": sum(sl for _, sl, _ in stalls) * 1e3,
                        "where": {w: sum(1 for *_, x in stalls if x == w)
                                  for w in ("retire", "admit", "other")},
                        "longest": [[round(s0, 3), round(sl * 1e3, 3), w]
                                    for s0, sl, w in sorted(stalls, key=lambda z: -z[1])[:5]],
                        "overlapping_gc": in_gc,
                        "gc_pauses": len(gc_pauses),
                        "gc_max_ms": max((gl for _, gl in gc_pauses), default=0.0) * 1e3,
                        "gc_off": bool(gc_off)}
        return st

    def stats(self, wall_s: float) -> Dict:
        import numpy as np
        done = [r for r in self.requests if r.status == "done"]
        lat = np.array([r.latency for r in done]) * 1e3 if done else np.zeros(1)
        per = {}
        for g in self.pools:
            lg = np.array([r.latency for r in done if r.grid == g]) * 1e3
            if len(lg):
                per[str(g)] = {"n": int(len(lg)), "p50_ms": float(np.percentile(lg, 50)),
                               "p99_ms": float(np.percentile(lg, 99))}
        # where the time of a request goes: waiting to be taken in and
        # admitted (queue), the launch call (launch), and the device work until
        # the server saw it finish (complete); and the same parts averaged over
        # the requests slower than the p99 latency
        parts = {}
        if done:
            q = np.array([r.t_launch - r.t_arrive for r in done]) * 1e3
            la = np.array([r.t_issued - r.t_launch for r in done]) * 1e3
            co = np.array([r.t_done - r.t_issued for r in done]) * 1e3
            tail = lat > np.percentile(lat, 99)
            for name, v in (("queue", q), ("launch", la), ("complete", co)):
                parts[name] = {"p50_ms": float(np.percentile(v, 50)),
                               "p99_ms": float(np.percentile(v, 99)),
                               "tail_mean_ms": float(v[tail].mean()) if tail.any() else 0.0}
        return {
            "requests": len(self.requests), "done": len(done), "parts": parts,
            "failed": sum(r.status == "failed" for r in self.requests),
            "rejected": sum(r.status == "rejected" for r in self.requests),
            "wall_s": wall_s, "throughput_rps": len(done) / wall_s if wall_s > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "windows": self.windows_launched,
            "mean_window": len(done) / max(1, self.windows_launched),
            "peak_windows_in_flight": self.peak_windows,
            "peak_bytes_in_flight": self.peak_bytes, "per_grid": per,
        }


def poisson_trace(rate_hz: float, seconds: float, ngrids: int, seed: int = 1):
    """Open-loop Poisson arrivals, each on a uniformly chosen grid, with a
    per-request seed."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    n = int(rng.poisson(rate_hz * seconds))
    t = np.sort(rng.uniform(0.0, seconds, n))
    g = rng.integers(0, ngrids, n)
    s = rng.integers(0, 2 ** 62, n)
    return list(zip(t.tolist(), g.tolist(), s.tolist()))


class GpuExecutor(Executor):
    """Slot pools of resident grids on the current GPU, one stream per grid."""

    def __init__(self, grids: Sequence, capacities: Sequence[int], tile_be: int = 256):
        import torch
        from . import acopf as A
        self.A = A
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.pool = []
        for g, cap in zip(grids, capacities):
            net = A.acopf_net_create(g)
            b = A.acopf_batch_create([net] * int(cap), tile_be=tile_be, grid_mult=0, xcd_group=0,
                                     no_graph=1)
            nx, nc = int(b.x_off[-1]), int(b.c_off[-1])
            nj, nh = int(b.j_off[-1]), int(b.h_off[-1])
            z = lambda n: torch.zeros(n, dtype=torch.float64, device=self.dev)
            bufs = dict(x=z(nx), lam=z(nc), sigma=torch.ones(cap, dtype=torch.float64, device=self.dev),
                        f=z(cap), gf=z(nx), c=z(nc), jac=z(nj), hess=z(nh))
            seeds = torch.zeros(cap, dtype=torch.int64, device=self.dev)
            pinned = torch.zeros(cap, dtype=torch.int64, pin_memory=True)
            bounds = (float(g.gen_pmin[0]) if g.ngen else 0.0, float(g.gen_pmax[0]) if g.ngen else 0.0,
                      float(g.gen_qmin[0]) if g.ngen else 0.0, float(g.gen_qmax[0]) if g.ngen else 0.0)
            per_slot = 8 * (2 * net.n + 2 * net.m + 1 + net.nnz_jac + net.nnz_hess) + 16
            stream = torch.cuda.Stream()
            # the seeded window's one library call, its pointer arguments
            # marshalled once: (batch, first, count, seeds, bounds, buffers, stream)
            vp = lambda t: ctypes.c_void_p(t.data_ptr())
            fast = ([b.handle], [ctypes.c_double(v) for v in bounds],
                    [vp(bufs[k]) for k in ("x", "lam", "sigma", "f", "gf", "c", "jac", "hess")]
                    + [ctypes.c_void_p(stream.cuda_stream)])
            self.pool.append(dict(net=net, batch=b, bufs=bufs, seeds=seeds, pinned=pinned,
                                  bounds=bounds, cap=int(cap), stream=stream,
                                  slot_bytes=per_slot, fast=fast))

    def grids(self):
        return list(range(len(self.pool)))

    def capacity(self, grid):
        return self.pool[grid]["cap"]

    def slot_bytes(self, grid):
        return self.pool[grid]["slot_bytes"]

    def check_inputs(self, grid, x, lam):
        net = self.pool[grid]["net"]
        if len(x) != net.n or len(lam) != net.m:
            raise ValueError(f"grid {grid} takes x of {net.n} and lam of {net.m} entries")

    def launch(self, grid, first, seeds, inputs=None):
        """Draw the window's iterates from the seeds, overwrite the slots whose
        request brought its own (x, lam, sigma), evaluate; returns the
        completion event.  A window of seeded requests only is one library
        call (acopf_batch_serve_window), the seeds in its launch arguments."""
        import torch
        P = self.pool[grid]
        k = len(seeds)
        if not inputs or all(inp is None for inp in inputs):
            head, bounds, tail = P["fast"]
            arr = (ctypes.c_uint64 * k)(*[s & ((1 << 63) - 1) for s in seeds])
            rc = self.A.lib().acopf_batch_serve_window(*head, first, k, arr, *bounds, *tail)
            if rc:
                raise self.A.AcopfError(rc, self.A.lib().acopf_last_error().decode())
            ev = torch.cuda.Event()
            ev.record(P["stream"])
            return ev
        P["pinned"][first:first + k] = torch.tensor([s & ((1 << 63) - 1) for s in seeds],
                                                    dtype=torch.int64)
        st = P["stream"]
        caller = torch.cuda.current_stream()
        with torch.cuda.stream(st):
            P["seeds"][first:first + k].copy_(P["pinned"][first:first + k], non_blocking=True)
            b, B = P["batch"], P["bufs"]
            self.A.acopf_batch_draw_iterates(b, first, k, P["seeds"], P["bounds"], B["x"],
                                             B["lam"], st)
            B["sigma"][first:first + k].fill_(1.0)
            for i, inp in enumerate(inputs or ()):
                if inp is None:
                    continue
                s = first + i
                x, lam, sigma = inp
                on_device = any(isinstance(t, torch.Tensor) and t.is_cuda for t in (x, lam))
                if on_device:
                    st.wait_stream(caller)  # work that produced the caller's tensors
                B["x"][int(b.x_off[s]):int(b.x_off[s + 1])].copy_(
                    torch.as_tensor(x, dtype=torch.float64), non_blocking=True)
                B["lam"][int(b.c_off[s]):int(b.c_off[s + 1])].copy_(
                    torch.as_tensor(lam, dtype=torch.float64), non_blocking=True)
                B["sigma"][s:s + 1].fill_(sigma)
            self.A.acopf_batch_eval_range(b, first, k, B["x"], B["sigma"], B["lam"], B["f"],
                                          B["gf"], B["c"], B["jac"], B["hess"],
                                          self.A.ACOPF_ALL, st)
            ev = torch.cuda.Event()
            ev.record(st)
        return ev

    def done(self, handle):
        return handle.query()

    def collect(self, grid, slot):
        """Device copies of one slot's outputs.  The copies run on the grid's
        stream (so later windows there cannot overwrite the slot first); the
        copy tensors belong to the caller's current stream, and the allocator
        is told that the grid's stream uses them too, so their memory is not
        handed out again before the copies have run."""
        import torch
        P = self.pool[grid]
        b, B = P["batch"], P["bufs"]
        st = P["stream"]
        srcs = {"f": B["f"][slot:slot + 1],
                "grad_f": B["gf"][int(b.x_off[slot]):int(b.x_off[slot + 1])],
                "c": B["c"][int(b.c_off[slot]):int(b.c_off[slot + 1])],
                "jac_val": B["jac"][int(b.j_off[slot]):int(b.j_off[slot + 1])],
                "hess_val": B["hess"][int(b.h_off[slot]):int(b.h_off[slot + 1])]}
        out = {k: torch.empty_like(v) for k, v in srcs.items()}
        # the caller's stream may have used this memory before: copy after it
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            for k, v in srcs.items():
                out[k].copy_(v, non_blocking=True)
                out[k].record_stream(st)
        return out

    def mark(self, grid):
        import torch
        ev = torch.cuda.Event()
        ev.record(self.pool[grid]["stream"])
        return ev

    def fetch(self, grid, slot):
        """Host copies of one slot's outputs (tests)."""
        P = self.pool[grid]
        b, B = P["batch"], P["bufs"]
        P["stream"].synchronize()
        sl = lambda t, o: t[int(o[slot]):int(o[slot + 1])].cpu().numpy()
        return {"x": sl(B["x"], b.x_off), "lam": sl(B["lam"], b.c_off),
                "f": float(B["f"][slot].cpu()), "grad_f": sl(B["gf"], b.x_off),
                "c": sl(B["c"], b.c_off), "jac_val": sl(B["jac"], b.j_off),
                "hess_val": sl(B["hess"], b.h_off)}

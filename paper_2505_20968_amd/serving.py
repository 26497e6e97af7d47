"""Continuous-batching serving loop for forward Stokes solves.

Requests (an atom, grids and a seeded atmosphere) arrive over time.  The
server admits queued requests in arrival order while the device-memory budget
(computed per request by ``trap_footprint``) and the slot limit allow; each
admitted request gets its own context and HIP stream, on which its precompute
and the start of its GMRES solve are enqueued without waiting.  Requests whose
precompute has finished advance together through ``trap_gmres_step_batch``:
one step enqueues the next unit of every such request's solve before waiting,
so their device work overlaps (and their FP32 operator applies share
launches), and the host synchronises at most twice per step for the whole
batch; precomputes of newly admitted requests run on the device meanwhile.  A
finished request releases its memory at once, so requests that arrived while
others were on the GPU join the batch as soon as memory frees up.  Krylov
state stays on the device for the whole solve.

The scheduling policy lives in :class:`Scheduler`, which drives an abstract
backend; :class:`DeviceBackend` is the GPU backend over the C ABI.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, List, Optional, Sequence

TRAP_ENOMEM = -2
TRAP_EDEVICE = -3


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    problem: Any
    admitted: Optional[float] = None
    done: Optional[float] = None
    status: Optional[int] = None
    stats: Optional[dict] = None
    result: Any = None        # backend result (the emergent Stokes profiles on the device backend)

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class Scheduler:
    """Arrival-order admission under a memory budget and a slot limit, one
    batched step per iteration, immediate release of finished requests.

    backend must provide ``footprint(problem) -> bytes``, ``admit(problem) ->
    handle``, ``step(handles) -> list of status`` (1 running, else final status)
    and ``finish(handle) -> (status, stats, result)``.  An admit that raises
    ends that request only (status: the exception's ``code``, else
    TRAP_EDEVICE); the backend releases what it had built for it.  A backend
    with ``device_free() -> bytes`` and ``reserve`` (bytes) is also held to
    what the device has free: a request waits until the device keeps
    ``reserve`` free beside it (room for the runtime's own allocations, kernel
    scratch among them), and is rejected when nothing runs and it still does
    not fit."""

    def __init__(self, backend, mem_budget: int, max_active: int = 16,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.backend = backend
        self.mem_budget = int(mem_budget)
        self.max_active = int(max_active)
        self.clock = clock
        self.sleep = sleep
        self.peak_used = 0
        self.peak_active = 0
        self.steps = 0
        self.time_admit = 0.0     # host seconds spent in backend.admit / step / finish
        self.time_step = 0.0
        self.time_finish = 0.0

    def run(self, requests: Sequence[Request]) -> List[Request]:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        active = []               # (request, handle, bytes)
        used = 0
        t0 = self.clock()
        while pending or queue or active:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            while queue and len(active) < self.max_active:
                req = queue[0]
                need = int(self.backend.footprint(req.problem))
                if need > self.mem_budget:            # can never fit: reject
                    queue.popleft()
                    req.status = TRAP_ENOMEM
                    req.admitted = req.done = self.clock() - t0
                    continue
                if used + need > self.mem_budget:     # wait for memory (arrival order is kept)
                    break
                if hasattr(self.backend, "device_free"):
                    if self.backend.device_free() - need < getattr(self.backend, "reserve", 0):
                        if active:                    # finished requests give memory back
                            break
                        queue.popleft()               # nothing runs: it cannot fit now
                        req.status = TRAP_ENOMEM
                        req.admitted = req.done = self.clock() - t0
                        continue
                queue.popleft()
                req.admitted = self.clock() - t0
                ta = self.clock()
                try:
                    handle = self.backend.admit(req.problem)
                except Exception as e:       # the request fails alone; the stream goes on
                    self.time_admit += self.clock() - ta
                    req.status = int(getattr(e, "code", TRAP_EDEVICE))
                    req.stats = {"error": str(e)}
                    req.done = self.clock() - t0
                    continue
                self.time_admit += self.clock() - ta
                active.append((req, handle, need))
                used += need
                self.peak_used = max(self.peak_used, used)
            self.peak_active = max(self.peak_active, len(active))
            if not active:
                if pending:
                    self.sleep(max(0.0, min(pending[0].arrival - (self.clock() - t0), 0.01)))
                continue
            ta = self.clock()
            status = self.backend.step([h for _, h, _ in active])
            self.time_step += self.clock() - ta
            self.steps += 1
            keep = []
            for (req, handle, need), s in zip(active, status):
                if s == 1:
                    keep.append((req, handle, need))
                    continue
                ta = self.clock()
                req.status, req.stats, req.result = self.backend.finish(handle)
                self.time_finish += self.clock() - ta
                req.done = self.clock() - t0
                used -= need
            active = keep
        return list(requests)


class DeviceBackend:
    """GPU backend: one context and HIP stream per request, batched GMRES steps."""

    def __init__(self, device: int = 0, precision: str = "mixed", tol: float = 1e-8, restart: int = 40,
                 inner_tol: float = 1e-7, max_outer: int = 10, max_iters: int = 2000, precond_sweeps: int = 0):
        import torch
        from .trap import TRAP_FP32, TRAP_FP64, footprint
        self.torch = torch
        self.device = device
        self.mixed = precision == "mixed"
        self.store = 3 if self.mixed else 1
        self.precond = int(precond_sweeps)
        self.opts = dict(tol=tol, restart=restart, max_iters=max_iters, max_outer=max_outer,
                         inner=TRAP_FP32 if self.mixed else TRAP_FP64, inner_tol=inner_tol, zero_guess=True,
                         precond_sweeps=self.precond)
        self._footprint = footprint
        self.admit_parts = {"context": 0.0, "set_problem": 0.0, "precompute": 0.0, "begin": 0.0}
        # device memory kept free beside the admitted requests (5 % of the device)
        self.reserve = int(0.05 * torch.cuda.mem_get_info(device)[1])

    def device_free(self) -> int:
        return int(self.torch.cuda.mem_get_info(self.device)[0])

    def footprint(self, problem) -> int:
        # library allocations plus the solution vector held by the caller
        n = 4 * problem.n_z * problem.n_dir * problem.n_nu
        return self._footprint(problem, self.store | (4 if self.precond else 0)) + 8 * n

    def admit(self, problem):
        """Set up the request and enqueue its precompute and the start of its
        solve on its own stream; returns without waiting for the device."""
        from .trap import Context
        torch = self.torch
        t0 = time.perf_counter()
        stream = torch.cuda.Stream(self.device)
        ctx = Context(self.device, stream)
        try:
            t1 = time.perf_counter()
            ctx.set_problem(problem)
            t2 = time.perf_counter()
            ctx.precompute(self.store)
            if self.precond:
                ctx.precompute_preconditioner()
            t3 = time.perf_counter()
            with torch.cuda.stream(stream):
                x = torch.zeros(ctx.shape, dtype=torch.float64, device=f"cuda:{self.device}")
            ctx.gmres_begin(x, **self.opts)
        except Exception:
            ctx.close()                   # what the failed admission allocated goes back at once
            raise
        ready = torch.cuda.Event()
        ready.record(stream)
        t4 = time.perf_counter()
        for k, dt in zip(self.admit_parts, (t1 - t0, t2 - t1, t3 - t2, t4 - t3)):
            self.admit_parts[k] += dt
        return {"ctx": ctx, "x": x, "stream": stream, "ready": ready, "is_ready": False}

    def step(self, handles):
        """One batched GMRES step over the requests whose precompute has
        finished; the others keep running on the device meanwhile (status 1).
        When none has finished, wait for the oldest."""
        from .trap import gmres_step_batch
        for h in handles:
            if not h["is_ready"] and h["ready"].query():
                h["is_ready"] = True
        if not any(h["is_ready"] for h in handles):
            handles[0]["ready"].synchronize()
            handles[0]["is_ready"] = True
        live = [h for h in handles if h["is_ready"]]
        st = iter(gmres_step_batch([h["ctx"] for h in live]))
        return [next(st) if h["is_ready"] else 1 for h in handles]

    def finish(self, handle):
        from .trap import TrapError
        ctx, x = handle["ctx"], handle["x"]
        try:
            stats = ctx.gmres_end(raise_on_noconv=False)
            em = ctx.emergent(x)
        except TrapError as e:            # the request fails alone
            ctx.close()
            return int(e.code), {"error": str(e)}, None
        ctx.close()
        return stats["status"], stats, em


def serve(requests: Sequence[Request], precision: str = "mixed", mem_budget: Optional[int] = None,
          max_active: int = 16, device: int = 0, **solver) -> dict:
    """Run a request stream on the device; returns the requests and summary figures."""
    import torch
    backend = DeviceBackend(device, precision, **solver)
    if mem_budget is None:
        free, _ = torch.cuda.mem_get_info(device)
        mem_budget = int(0.8 * free)
    sched = Scheduler(backend, mem_budget, max_active)
    t0 = time.perf_counter()
    out = sched.run(requests)
    wall = time.perf_counter() - t0
    ok = [r for r in out if r.status == 0]
    lat = sorted(r.latency for r in ok)

    def pct(q):
        if not lat:
            return None
        k = (len(lat) - 1) * q
        lo = int(k)
        hi = min(lo + 1, len(lat) - 1)
        return lat[lo] + (lat[hi] - lat[lo]) * (k - lo)

    return {"requests": out, "wall_s": wall, "solves_per_s": len(ok) / wall if wall > 0 else 0.0,
            "n_ok": len(ok), "n_rejected": sum(1 for r in out if r.status == TRAP_ENOMEM),
            "n_failed": sum(1 for r in out if r.status not in (0, TRAP_ENOMEM)),
            "p50_s": pct(0.5), "p99_s": pct(0.99), "peak_active": sched.peak_active,
            "peak_bytes": sched.peak_used, "steps": sched.steps,
            "host_s": {"admit": sched.time_admit, "step": sched.time_step, "finish": sched.time_finish,
                       "admit_parts": dict(backend.admit_parts)}}

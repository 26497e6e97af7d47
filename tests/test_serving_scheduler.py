"""Host logic of the serving loop (no GPU): admission in arrival order under a
memory budget and a slot limit, rejection of requests that can never fit,
release on completion, latency accounting."""
from paper_2505_20968_amd.serving import Request, Scheduler, TRAP_ENOMEM


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-3)


class FakeBackend:
    """Each request needs problem['steps'] batched steps; a step costs 1 s."""

    def __init__(self, clock):
        self.clock = clock
        self.live = {}
        self.log = []

    def footprint(self, p):
        return p["mem"]

    def admit(self, p):
        h = len(self.log)
        self.live[h] = p["steps"]
        self.log.append(("admit", p["id"], self.clock()))
        return h

    def step(self, handles):
        self.clock.t += 1.0
        out = []
        for h in handles:
            self.live[h] -= 1
            out.append(1 if self.live[h] > 0 else 0)
        return out

    def finish(self, h):
        del self.live[h]
        return 0, {"steps": "done"}, h


def _run(reqs, budget, max_active):
    clock = FakeClock()
    be = FakeBackend(clock)
    s = Scheduler(be, budget, max_active, clock=clock, sleep=clock.sleep)
    out = s.run(reqs)
    return s, be, out


def test_budget_and_slots_are_respected():
    reqs = [Request(i, 0.0, {"id": i, "mem": 40, "steps": 3}) for i in range(6)]
    s, be, out = _run(reqs, budget=100, max_active=4)
    assert all(r.status == 0 for r in out)
    assert s.peak_used <= 100 and s.peak_active == 2          # memory allows two at a time
    s, be, out = _run([Request(i, 0.0, {"id": i, "mem": 10, "steps": 3}) for i in range(6)], 100, 4)
    assert s.peak_active == 4


def test_never_fitting_request_is_rejected_and_others_run():
    reqs = [Request(0, 0.0, {"id": 0, "mem": 500, "steps": 2}),
            Request(1, 0.0, {"id": 1, "mem": 50, "steps": 2})]
    s, be, out = _run(reqs, budget=100, max_active=4)
    assert out[0].status == TRAP_ENOMEM and out[0].result is None
    assert out[1].status == 0


def test_late_arrivals_join_running_batch_when_memory_frees():
    reqs = [Request(0, 0.0, {"id": 0, "mem": 60, "steps": 10}),
            Request(1, 0.0, {"id": 1, "mem": 40, "steps": 2}),
            Request(2, 1.5, {"id": 2, "mem": 40, "steps": 2})]
    s, be, out = _run(reqs, budget=100, max_active=8)
    r0, r1, r2 = out
    # request 2 arrives while 0 and 1 run, waits for 1 to free its memory,
    # and finishes before the long request 0
    assert r2.admitted >= r1.done and r2.admitted >= r2.arrival
    assert r2.done < r0.done
    assert s.peak_used <= 100


def test_arrival_order_is_kept_and_latency_is_measured():
    reqs = [Request(i, 0.5 * i, {"id": i, "mem": 30, "steps": 1 + i % 3}) for i in range(8)]
    s, be, out = _run(reqs, budget=60, max_active=8)
    adm = [r.admitted for r in sorted(out, key=lambda r: r.arrival)]
    assert adm == sorted(adm)
    for r in out:
        assert r.status == 0 and r.latency == r.done - r.arrival and r.latency > 0


class FailingBackend(FakeBackend):
    """Admission of requests marked 'bad' raises, as a set-up or precompute
    error of the library does (an exception carrying the status code)."""

    class Failure(RuntimeError):
        def __init__(self, code):
            super().__init__(f"admission failed with {code}")
            self.code = code

    def admit(self, p):
        if p.get("bad"):
            self.log.append(("fail", p["id"], self.clock()))
            raise self.Failure(-1)
        return super().admit(p)


def test_an_admission_failure_ends_that_request_only():
    clock = FakeClock()
    be = FailingBackend(clock)
    s = Scheduler(be, 100, 4, clock=clock, sleep=clock.sleep)
    reqs = [Request(i, 0.0, {"id": i, "mem": 40, "steps": 2, "bad": i == 1}) for i in range(4)]
    out = s.run(reqs)
    bad = out[1]
    assert bad.status == -1 and bad.done is not None and "admission failed" in bad.stats["error"]
    assert all(r.status == 0 for r in out if r.rid != 1)
    # its memory was never held: two requests fit the budget at a time, and the
    # failed one did not delay the others
    assert s.peak_used <= 100
    assert [e[1] for e in be.log if e[0] == "admit"] == [0, 2, 3]
    assert max(r.done for r in out) <= 4.0 + 1e-9


class DeviceHoldingBackend(FakeBackend):
    """A device of `total` bytes of which `held_elsewhere` are taken by others
    (memory no footprint counts); it keeps `reserve` free beside the requests."""

    def __init__(self, clock, total, held_elsewhere, reserve):
        super().__init__(clock)
        self.total, self.held_elsewhere, self.reserve = total, held_elsewhere, reserve
        self.mem = {}

    def admit(self, p):
        h = super().admit(p)
        self.mem[h] = p["mem"]
        assert self.device_free() >= self.reserve            # never admitted past the reserve
        return h

    def finish(self, h):
        del self.mem[h]
        return super().finish(h)

    def device_free(self):
        return self.total - self.held_elsewhere - sum(self.mem.values())


def test_device_free_memory_and_reserve_are_respected():
    """The budget alone would admit all four at once; the device has less free
    than the budget assumes, so requests wait for finished ones, and one that
    cannot fit beside the reserve even on an idle device is rejected."""
    clock = FakeClock()
    be = DeviceHoldingBackend(clock, total=200, held_elsewhere=60, reserve=20)
    reqs = [Request(i, 0.0, {"id": i, "mem": 50, "steps": 2}) for i in range(4)]
    reqs.append(Request(4, 0.0, {"id": 4, "mem": 130, "steps": 1}))      # 200 - 60 - 130 < 20
    s = Scheduler(be, mem_budget=1000, max_active=8, clock=clock, sleep=clock.sleep)
    out = s.run(reqs)
    assert [r.status for r in out[:4]] == [0, 0, 0, 0]
    assert out[4].status == TRAP_ENOMEM
    assert s.peak_active == 2                                 # 140 free - 2 x 50 leaves the 20 reserve

"""Host logic of the solve server, on the CPU: the device calls are replaced
by stand-ins that complete instantly, so only the scheduling is exercised
(admission by footprint within the budget, arrival order, every request
finishing, slots released)."""
import types

import pytest

from paper_2602_05900_amd import serve, workloads


class FakeEvent:
    def record(self, stream):
        pass

    def query(self):
        return True


class FakeSolve:
    live = 0

    def __init__(self, **kw):
        self.kw = kw
        self.steps = 0
        self.polls = 0
        FakeSolve.live += 1

    def coarse_grain(self, n):
        self.steps += n
        return self

    def step_begin(self, exchange=True, extra=0):
        # steps of the small dims are enqueued whole; later ones need polls
        if self.steps < 2:
            self.steps += 1
            return False
        self.polls = 3
        return True

    def step_poll(self):
        from paper_2602_05900_amd import binding
        if self.polls == 0:
            return binding.POLL_IDLE
        self.polls -= 1
        if self.polls == 2:
            return binding.POLL_RUNNING
        if self.polls == 1:
            return binding.POLL_PASSES
        self.steps += 1
        return binding.POLL_STEPPED

    def coarse_grain_async(self, n, exchange=True, extra=0):
        self.steps += n
        self.busy = 2

    def async_busy(self):
        self.busy = max(self.busy - 1, 0)
        return self.busy > 0

    def log_z(self):
        return 1.0 + self.kw["temperature"] * 1e-3 + self.steps * 1e-6

    def stage_times(self):
        return {}, 0

    def set_timing(self, on=True):
        pass

    def close(self):
        FakeSolve.live -= 1


@pytest.fixture
def fake_device(monkeypatch):
    import torch
    monkeypatch.setattr(serve.binding, "load", lambda: None)
    monkeypatch.setattr(serve.binding, "Solve", FakeSolve)
    monkeypatch.setattr(serve.binding, "coarse_grain_batch",
                        lambda solves, n: [s.coarse_grain(n) for s in solves])
    # footprint grows like D^5 (bytes), as the real sizing does
    monkeypatch.setattr(serve.binding, "workspace_bytes",
                        lambda **kw: 16 * kw["dmax"] ** 5 + 1000 * kw["max_steps"])
    monkeypatch.setattr(torch.cuda, "Stream", lambda device=None: types.SimpleNamespace(cuda_stream=0))
    monkeypatch.setattr(torch.cuda, "Event", FakeEvent)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda device=None: None)
    monkeypatch.setattr(torch, "empty", lambda n, dtype=None, device=None: types.SimpleNamespace(numel=lambda: n))
    FakeSolve.live = 0
    yield


def test_admission_respects_budget_and_completes_everything(fake_device):
    reqs = workloads.request_stream(rate_hz=200.0, duration_s=0.5, seed=3)
    budget = 16 * 48 ** 5 * 2 + 10 ** 6      # room for about two D=48 solves
    srv = serve.Server(slots=6, budget=budget, precision="fp64", device="cpu")
    done = srv.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    assert {c.rid for c in done} == {r.rid for r in reqs}
    assert all(c.lnz_per_site > 0 for c in done)
    # the budget is never exceeded, and memory and slots are all given back
    assert max(u for _, _, u in srv.admission_log) <= budget
    assert srv.peak_in_use <= budget
    assert srv.in_use == 0 and len(srv.free_streams) == 6 and FakeSolve.live == 0
    # admission in arrival order
    order = [rid for rid, _, _ in srv.admission_log]
    assert order == sorted(order)
    # every solve was advanced by exactly its step count
    for c in done:
        r = reqs[c.rid]
        assert c.nsteps == r.nsteps and abs(c.lnz_per_site - (1.0 + r.temperature * 1e-3 + r.nsteps * 1e-6)) < 1e-12


def test_polled_server_takes_every_step(fake_device):
    """The host-polled form: every solve ends with exactly its step count,
    whole steps and polled steps mixed, and nothing is left pending."""
    reqs = workloads.request_stream(rate_hz=200.0, duration_s=0.3, seed=5)
    srv = serve.Server(slots=4, budget=1 << 40, precision="fp64", device="cpu", stepping="polled")
    done = srv.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    for c in done:
        r = reqs[c.rid]
        assert abs(c.lnz_per_site - (1.0 + r.temperature * 1e-3 + r.nsteps * 1e-6)) < 1e-12
    assert srv.in_use == 0 and FakeSolve.live == 0


def test_engine_server_takes_every_step(fake_device):
    reqs = workloads.request_stream(rate_hz=200.0, duration_s=0.3, seed=6)
    srv = serve.Server(slots=4, budget=1 << 40, precision="fp64", device="cpu", stepping="engine")
    done = srv.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    for c in done:
        r = reqs[c.rid]
        assert abs(c.lnz_per_site - (1.0 + r.temperature * 1e-3 + r.nsteps * 1e-6)) < 1e-12
    assert srv.in_use == 0 and FakeSolve.live == 0
    with pytest.raises(ValueError):
        serve.Server(slots=1, device="cpu", stepping="sometimes")


def test_hybrid_server_takes_every_step(fake_device):
    """Small solves driven by the progress thread, large ones by whole steps,
    in one server."""
    reqs = workloads.request_stream(rate_hz=200.0, duration_s=0.3, seed=7)
    assert {r.dmax <= 32 for r in reqs} == {True, False}
    srv = serve.Server(slots=4, budget=1 << 40, precision="fp64", device="cpu", stepping="hybrid")
    done = srv.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    for c in done:
        r = reqs[c.rid]
        assert abs(c.lnz_per_site - (1.0 + r.temperature * 1e-3 + r.nsteps * 1e-6)) < 1e-12
    assert srv.in_use == 0 and FakeSolve.live == 0


def test_request_larger_than_budget_is_rejected(fake_device):
    reqs = [workloads.Request(rid=0, arrival=0.0, model="ising", q=2, temperature=2.0, dmax=48, nsteps=20)]
    srv = serve.Server(slots=2, budget=1000, device="cpu")
    with pytest.raises(ValueError):
        srv.run(reqs, realtime=False)


def test_request_stream_recipe():
    reqs = workloads.request_stream(rate_hz=50.0, duration_s=60.0)
    assert 2700 < len(reqs) < 3300                       # Poisson(3000)
    assert all(0 <= r.arrival < 60.0 for r in reqs)
    assert {r.model for r in reqs} == {"ising", "potts"}
    assert {r.dmax for r in reqs} <= {16, 24, 32, 48}
    assert min(r.nsteps for r in reqs) >= 20 and max(r.nsteps for r in reqs) <= 40
    for r in reqs:
        tc = workloads.critical_temperature(r.model, r.q)
        assert 0.5 * tc <= r.temperature <= 1.5 * tc
    # seeded: the same stream every time
    again = workloads.request_stream(rate_hz=50.0, duration_s=60.0)
    assert [(r.arrival, r.temperature) for r in again[:50]] == [(r.arrival, r.temperature) for r in reqs[:50]]


def test_percentiles():
    xs = list(range(1, 101))
    assert serve.percentile(xs, 50) == pytest.approx(50.5)
    assert serve.percentile(xs, 99) == pytest.approx(99.01)
    s = serve.summarize([], 1.0)
    assert s["solves"] == 0

"""The benchmark's command-line contract on the host (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1",
                        "--warmup", "0"], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


class _FakeSolve:
    """Stands in for binding.Solve in the roofline leg: 30 steps whose Y
    stage takes 4 ms at the steady dims."""

    def __init__(self, **kw):
        self.kw = kw
        self.n = 0

    def set_timing(self, on=True):
        pass

    def coarse_grain(self, n, exchange=True):
        self.n += n
        return self

    def log_z(self):
        return 1.0

    def step_stage_times(self):
        from paper_2602_05900_amd import accounting, binding
        d = self.kw["dmax"]
        out = []
        for dims in accounting.step_dims(2, 2, d, self.n):
            ms = {k: 0.1 for k in binding.STAGES}
            ms["y"] = 4.0 if dims == (d, d, d) else 0.5
            out.append((dims, ms))
        return out

    def close(self):
        pass


def _fake_server_class(calls):
    from paper_2602_05900_amd import accounting, serve

    class FakeServer:
        def __init__(self, slots=8, budget=0, depth=2, precision="fp64", device="cuda:0", timing=False,
                     stepping="whole"):
            self.precision = precision
            self.timing = timing
            self.peak_in_use = self.in_use = 0
            self.unfinished = []

        def run(self, requests, realtime=True, progress=None, horizon=None):
            calls.append((self.precision, [r.rid for r in requests], horizon))
            out = []
            for i, r in enumerate(requests):
                # ln Z / N of a fake solve: a smooth function of T, shifted by precision
                lnz = 1.0 / r.temperature + (1e-9 if self.precision != "fp64" else 0.0)
                out.append(serve.Completed(
                    rid=r.rid, model=r.model, q=r.q, temperature=r.temperature, dmax=r.dmax, nsteps=r.nsteps,
                    precision=self.precision, lnz_per_site=lnz, arrival=r.arrival, admitted=0.01 * i,
                    finished=0.01 * i + 0.2, footprint=1, flops=accounting.solve_flops(r.q, r.dmax, r.nsteps),
                    stage_ms={"env": 1.0, "x": 1.0, "y": 10.0, "tp": 1.0} if self.timing else None))
            return out

    return FakeServer


def test_bench_line_with_the_drivers_flags_and_a_failing_leg(monkeypatch, capsys):
    """The bookkeeping of bench.main with --steps 20 --warmup 5 on the host:
    the device is replaced by a fake server and solve, one side leg is made
    to fail, and the line must still come out whole, with that leg's error
    recorded under its own key."""
    import importlib
    import math
    import torch
    sys.path.insert(0, ROOT)
    bench = importlib.import_module("bench")
    from paper_2602_05900_amd import binding, serve
    calls = []
    monkeypatch.setattr(serve, "Server", _fake_server_class(calls))
    monkeypatch.setattr(binding, "Solve", _FakeSolve)
    monkeypatch.setattr(torch.cuda, "set_device", lambda d: None)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)

    def broken(*a, **k):
        raise RuntimeError("planted failure of a side leg")
    monkeypatch.setattr(bench, "run_c5", broken)
    bench.main(["--steps", "20", "--warmup", "5", "--cpu-sample-steps", "2", "--no-observables", "--no-itebd",
                "--no-qchain"])
    line = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config"):
        assert key in line, key
    assert line["steps"] == 20 and line["warmup"] == 5 and line["n_gpus"] == 1
    assert line["value"] > 0 and math.isfinite(line["ms_per_step"])
    # the timed batch and the FP64 comparison cover the same requests
    timed = [c for c in calls if c[0] == "fp16x3" and len(c[1]) == 20]
    bf = [c for c in calls if c[0] == "bf16x6" and len(c[1]) == 20]
    fp64 = [c for c in calls if c[0] == "fp64" and len(c[1]) == 20]
    assert timed and bf and fp64 and timed[0][1] == bf[0][1] == fp64[0][1] == list(range(5, 25))
    cmp = line["fp64_comparison"]
    assert "error" not in cmp and abs(cmp["max_rel_df_headline_vs_this"] - 1e-9 / 0.5) < 1e-9
    assert "error" not in line["bf16x6_comparison"]
    # the roofline: steady launches only, algorithmic FLOPs over their mean time
    rf = line["roofline"]
    assert rf["bound"] == "mfma" and rf["unit"] == "TFLOP/s" and rf["peak"] == 2500.0
    assert rf["avg_launch_ms"] == 4.0 and rf["launches"] == 24
    assert abs(rf["achieved"] - 2 * 48 ** 7 / 4e-3 / 1e12) < 1e-6
    assert abs(rf["frac"] - rf["achieved"] / 2500.0) < 1e-12
    assert "traffic" in rf
    # the failing leg is recorded, the others are there
    assert line["c5"]["error"].startswith("RuntimeError: planted failure")
    assert "error" not in line["c2"]
    c4 = line["c4"]
    assert "error" not in c4 and [r["rate_hz"] for r in c4["runs"]] == [10.0, 50.0]
    assert all(c[2] is not None for c in calls if c[2] is not None)
    cpu = line["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["unit"] == "TFLOP/s" and cpu["value"] > 0 and cpu["cores"] >= 1

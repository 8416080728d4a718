"""Serve a seeded Poisson stream of HOTRG solve requests and report latency.

Workload: arrivals at --rate requests/s for --seconds s; each request draws
its model from {Ising, 3-state Potts}, T uniform in [0.5, 1.5] x Tc(model),
D from {16, 24, 32, 48} and 20..40 steps (workloads.request_stream).  Prints
one JSON line: offered and served TFLOP/s, solves/s, p50/p99 latency
(arrival to completion) and service time, peak admitted footprint.

    python -m paper_2602_05900_amd.serve_bench [--rate 50] [--seconds 60] [--precision bf16x6]
    python -m paper_2602_05900_amd.serve_bench --sweep 5,10,15,20 --seconds 20

--sweep serves one stream per listed rate, one after another on the same
server (one JSON line each), to find the rate where latency stops being
service-dominated and becomes queue-dominated.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--precision", default="bf16x6")
    ap.add_argument("--sweep", default=None, help="comma-separated arrival rates (req/s) served in turn")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--budget-gb", type=int, default=160)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--stepping", default="whole", choices=["whole", "polled", "engine", "hybrid"])
    args = ap.parse_args()

    import torch
    from . import accounting, serve, workloads
    srv = serve.Server(slots=args.slots, budget=args.budget_gb << 30, precision=args.precision,
                       stepping=args.stepping)
    rates = [float(r) for r in args.sweep.split(",")] if args.sweep else [args.rate]
    for rate in rates:
        serve_stream(args, srv, rate, accounting, serve, workloads, torch)


def serve_stream(args, srv, rate, accounting, serve, workloads, torch):
    kw = {} if args.seed is None else {"seed": args.seed}
    reqs = workloads.request_stream(rate_hz=rate, duration_s=args.seconds, **kw)
    offered = sum(accounting.solve_flops(r.q, r.dmax, r.nsteps) for r in reqs) / args.seconds / 1e12
    srv.peak_in_use = srv.in_use

    def progress(now, done, total, active, queued):
        print(f"# {rate:g} req/s {now:6.1f} s: {done}/{total} done, {active} active, {queued} queued",
              file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = srv.run(reqs, realtime=True, progress=progress)
    wall = time.perf_counter() - t0
    summ = serve.summarize(done, wall)
    service = [c.finished - c.admitted for c in done]
    line = {
        "metric": "served HOTRG solves: p50/p99 latency and throughput",
        "workload": f"Poisson {rate:g} req/s for {args.seconds:g} s; Ising/Potts(q=3), T in [0.5,1.5] Tc, "
                    f"D in {{16,24,32,48}}, 20-40 steps",
        "precision": args.precision,
        "rate_hz": rate,
        "requests": len(reqs),
        "offered_tflops": offered,
        **summ,
        "p50_service_s": serve.percentile(service, 50),
        "p99_service_s": serve.percentile(service, 99),
        "slots": args.slots,
        "budget_gb": args.budget_gb,
        "peak_footprint_gb": srv.peak_in_use / 2 ** 30,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""HOTRG contraction throughput on one MI355X.

Workload (one "step" of this benchmark = one full HOTRG solve, every row of
the hot path): 2D Ising, J = 1, bond dimension D = 48, 30 alternating
coarse-graining steps, temperatures cycling through 16 evenly spaced values
in [2.0, 2.5].  The initial tensor is built from the temperature (128 bytes
of input); all intermediates stay in HBM.

The solves of the batch run concurrently (--concurrency of them in flight,
one HIP stream and workspace each) through the continuous-batching server.

value = algorithmic contraction FLOPs of the timed solves (O(D^7) order,
eigensolve excluded from the count but not from the time) / wall time of
the timed region, in the headline precision (default FP16X3: the D^7
product Y and the environment products with their operands split into two
FP16 terms of the value times a fixed power of two, 3 products, the X and
T' products split into three BF16 terms, 6 products, all with FP32
accumulation; eigensolve, normalisation
and ln Z in FP64).  Also reported: the same batch in BF16x6, FP32 and FP64, per-solve service time
p50/p99, per-stage GPU times from HIP events, |delta f| against the FP64
oracle's stored values for these temperatures, the roofline of the dominant
kernel (the steady-state Y product, 2 D^7 algorithmic FLOPs a launch,
measured on one solve running alone) and the FP64 CPU oracle on a bounded
sample.  Further workloads are measured and reported beside the headline
(not in `value`), each under its own key, where a failure is recorded as
{"error": ...} without dropping the line: a D = 24 FP64 scan of 64
temperatures with the finite-difference internal energy against Onsager
("c2"), served solves under Poisson arrivals ("c4"), one D = 64, 40-step
solve at Tc in BF16x6 and in FP64 ("c5"), two-sided truncation with
impurity observables, iTEBD chains and the quantum chain.

Stepping (--stepping for the headline batch and the served stream,
--latency-stepping for the one-solve-at-a-time legs C2, the observables and
the quantum chain): whole steps enqueue every eigensolver pass up to the cap, and a pass
after convergence exits at once; host-polled steps enqueue a step's
products once the eigensolve has stopped, either from the scheduler loop
("polled") or from the library's progress thread ("engine").  The results
are bitwise the same.  Measured, whole steps are faster with four solves in
flight and the engine is faster for one solve at a time, hence the defaults.

    python bench.py [--steps K] [--warmup W] [--precision fp64|fp32|bf16x3|bf16x6|fp16x3] [--concurrency C]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time
import traceback

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# dense MFMA peaks of the Y product's operand type (BF16 and FP16: 2.5 PFLOP/s)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0, "fp16x3": 2500.0}
TRAFFIC_PROFILE = {p: os.path.join(ROOT, "profiles", f"gemm_y_{p}_ising_d48_traffic.md") for p in ("bf16x6", "fp16x3")}
# bytes per element of Y's operands (X and the re-laid-out T)
ELEM_BYTES = {"fp64": 8, "fp32": 4, "bf16x3": 4, "bf16x6": 6, "fp16x3": 4}
# Y's output: FP32 in the split modes (its consumer splits it on load)
Y_OUT_BYTES = {"fp64": 8, "fp32": 4, "bf16x3": 4, "bf16x6": 4, "fp16x3": 4}
# MFMA products per algorithmic product in Y
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6, "fp16x3": 3}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3-split/f32acc", "bf16x6": "bf16x6-split/f32acc",
         "fp16x3": "fp16x3-split/f32acc (Y, environments), bf16x6-split/f32acc (X, T')"}


def measured_traffic(precision: str, dmax: int, nsteps: int):
    """HBM bytes per steady-state Y launch from the committed FETCH_SIZE /
    WRITE_SIZE summary of this workload, or None when there is none or when
    the product kernel's source has changed since the counters were taken."""
    path = TRAFFIC_PROFILE.get(precision)
    if path is None or dmax != 48 or nsteps != 30 or not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        key, sep, val = line.strip().partition(":")
        if sep and key in ("traffic_bytes_per_steady_launch", "kernel_source_sha256"):
            fields[key] = val.strip()
    src = os.path.join(ROOT, "paper_2602_05900_amd", "csrc", "gemm.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha or "traffic_bytes_per_steady_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_steady_launch"])


def fd_energy(temps, lnz):
    """u(T) = T^2 d(ln Z/N)/dT on a uniform grid: central differences inside,
    second-order one-sided differences at the ends."""
    h = temps[1] - temps[0]
    d = [0.0] * len(lnz)
    for i in range(1, len(lnz) - 1):
        d[i] = (lnz[i + 1] - lnz[i - 1]) / (2 * h)
    d[0] = (-3 * lnz[0] + 4 * lnz[1] - lnz[2]) / (2 * h)
    d[-1] = (3 * lnz[-1] - 4 * lnz[-2] + lnz[-3]) / (2 * h)
    return [t * t * g for t, g in zip(temps, d)]


def onsager_reference():
    path = os.path.join(ROOT, "tests", "golden", "onsager_ising.json")
    return json.load(open(path)) if os.path.exists(path) else None


def run_c2(serve, accounting, workloads, budget, stepping="engine"):
    """Ising, D = 24, 30 steps, FP64, 64 temperatures in [1.8, 2.8] one after
    another: throughput, f against Onsager, and the finite-difference internal
    energy against Onsager's u.  One solve at a time is latency-bound, so the
    steps are host-polled by the library's progress thread (`stepping`); the
    same scan with whole steps is timed beside it (bitwise the same ln Z)."""
    import numpy as np
    import torch
    temps = [float(t) for t in np.linspace(1.8, 2.8, 64)]
    reqs = [workloads.Request(rid=i, arrival=0.0, model="ising", q=2, temperature=t, dmax=24, nsteps=30)
            for i, t in enumerate(temps)]

    def scan(mode):
        server = serve.Server(slots=1, budget=budget, precision="fp64", device="cuda:0", stepping=mode)
        server.run(reqs[:1], realtime=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = server.run(reqs, realtime=False)
        return done, time.perf_counter() - t0

    done, wall = scan(stepping)
    lnz = [c.lnz_per_site for c in sorted(done, key=lambda c: c.rid)]
    u = fd_energy(temps, lnz)
    out = {"workload": "Ising J=1, D=24, 30 steps, FP64, T = linspace(1.8, 2.8, 64), one solve at a time",
           "stepping": stepping, "solves": len(done), "seconds": wall,
           "tflops": len(done) * accounting.solve_flops(2, 24, 30) / wall / 1e12}
    if stepping != "whole":
        done_w, wall_w = scan("whole")
        out["seconds_whole_steps"] = wall_w
        out["lnz_bitwise_equal_to_whole_steps"] = \
            [c.lnz_per_site for c in sorted(done_w, key=lambda c: c.rid)] == lnz
    ref = onsager_reference()
    if ref:
        g = ref["grid"]
        tc = ref["critical"]["temperature"]
        far = [abs(t - tc) > 0.1 for t in temps]
        df = [abs(a - b) / abs(b) for a, b in zip(lnz, g["lnz_per_site"])]
        du = [abs(a - b) for a, b in zip(u, g["energy"])]
        du_grid = [abs(a - b) for a, b in zip(g["energy_fd_of_exact_lnz"], g["energy"])]
        out.update({
            "max_rel_df_vs_onsager": max(df),
            "max_rel_df_vs_onsager_off_critical": max(d for d, f in zip(df, far) if f),
            "max_abs_du_fd_vs_onsager_off_critical": max(d for d, f in zip(du, far) if f),
            "max_abs_du_fd_vs_onsager": max(du),
            "fd_discretisation_error_off_critical": max(d for d, f in zip(du_grid, far) if f),
        })
    return out


def run_observables(binding, accounting, stepping="engine"):
    """Two-sided truncation with the magnetisation and bond-energy impurity
    tensors carried along.  (1) Ising, D = 24, 30 steps, FP64, 16
    temperatures of the D = 24 grid (every fourth of linspace(1.8, 2.8, 64)),
    field 1e-8 to select the ordered state below T_c, one solve at a time:
    throughput, the direct internal energy 2 <e_b> - h <m> against Onsager
    and <m> against Yang's spontaneous magnetisation.  (2) The same mode at
    D = 48 in BF16x6 at four temperatures: throughput.  One solve at a time:
    the steps are host-polled by the library's progress thread (`stepping`),
    and the D = 24 scan is timed with whole steps beside it."""
    import torch

    def advance(s, mode):
        if mode == "engine":
            s.coarse_grain_async(30)
        else:
            s.coarse_grain(30)
    ref = onsager_reference()
    g = ref["grid"] if ref else None
    idx = list(range(0, 64, 4))
    temps = [g["temperatures"][i] for i in idx] if g else [1.8 + i / 63.0 for i in idx]
    h = 1e-8
    nimp = 2
    out = {"workload": "Ising J=1, D=24, 30 steps, FP64, two-sided, observables m and e, h=1e-8, "
                       "T = linspace(1.8, 2.8, 64)[::4], one solve at a time"}
    s = binding.Solve(model="ising", q=2, temperature=temps[0], dmax=24, precision="fp64", max_steps=30,
                      field=h, two_sided=True, observables=("m", "e"))
    s.coarse_grain(30)
    s.observables()
    def scan(mode):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = []
        for t in temps:
            s.reset(model="ising", q=2, temperature=t, dmax=24, precision="fp64", max_steps=30, field=h,
                    two_sided=True, observables=("m", "e"))
            advance(s, mode)
            v = s.observables()
            res.append((t, s.log_z(), v["m"], v["e"]))
        return res, time.perf_counter() - t0

    res, wall = scan(stepping)
    flops = accounting.solve_flops(2, 24, 30, two_sided=True, nimp=nimp)
    out.update({"stepping": stepping, "solves": len(res), "seconds": wall,
                "tflops": len(res) * flops / wall / 1e12, "flops_per_solve": flops})
    if stepping != "whole":
        res_w, wall_w = scan("whole")
        out["seconds_whole_steps"] = wall_w
        out["results_bitwise_equal_to_whole_steps"] = res_w == res
    s.close()
    if g:
        tc = ref["critical"]["temperature"]
        du, dm, dmf = [], [], []
        for (t, _lnz, m, e), i in zip(res, idx):
            u = 2.0 * e - h * m
            far = abs(t - tc) > 0.1
            if far:
                du.append(abs(u - g["energy"][i]))
                dm.append(abs(m - g["magnetisation"][i]))
        out.update({"max_abs_du_direct_vs_onsager_off_critical": max(du),
                    "max_abs_dm_vs_yang_off_critical": max(dm),
                    "energy_direct": [2.0 * e - h * m for (_t, _l, m, e) in res],
                    "magnetisation": [m for (_t, _l, m, _e) in res]})
    # D = 48, BF16x6
    temps48 = [2.0, 2.2, 2.4, 2.5]
    s = binding.Solve(model="ising", q=2, temperature=temps48[0], dmax=48, precision="bf16x6", max_steps=30,
                      field=h, two_sided=True, observables=("m", "e"))
    s.coarse_grain(30)
    s.observables()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in temps48:
        s.reset(model="ising", q=2, temperature=t, dmax=48, precision="bf16x6", max_steps=30, field=h,
                two_sided=True, observables=("m", "e"))
        advance(s, stepping)
        s.observables()
    wall = time.perf_counter() - t0
    s.close()
    f48 = accounting.solve_flops(2, 48, 30, two_sided=True, nimp=nimp)
    out["d48_bf16x6"] = {"workload": "Ising J=1, D=48, 30 steps, BF16x6, two-sided, observables m and e, "
                                     "T in {2.0, 2.2, 2.4, 2.5}, one solve at a time",
                         "solves": len(temps48), "seconds": wall, "tflops": len(temps48) * f48 / wall / 1e12,
                         "flops_per_solve": f48}
    return out


def run_itebd(binding, workloads):
    """iTEBD of the S = 1/2 antiferromagnetic Heisenberg chain (the paper's
    iTEBD workload), FP64, random initial states: (1) 512 chains (two per
    CU) at D_b = 30 for 10,000 bond updates at tau = 0.01 (aggregate
    updates/s and the energy per site against the Bethe value); (2) time per
    bond update against D_b for one chain and for 512 chains (1,000 updates
    each), with the fitted exponent x of time ~ D_b^x."""
    import math
    import numpy as np
    import torch
    h = workloads.heisenberg_bond()
    bethe = 0.25 - math.log(2.0)
    out = {"workload": "S=1/2 AF Heisenberg chain, FP64, random initial states, one workgroup per chain, "
                       "two chains per CU"}
    from paper_2602_05900_amd import chain_bench
    chi, batch, nup = 30, 512, 10000
    c = binding.Chains(h, workloads.random_chain_states(batch, chi, seed=2026), chi)
    c.evolve(0.1, 200)
    c.energies()
    sw0, rot0 = c.work()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(c.stream)
    c.evolve(0.01, nup)
    ev1.record(c.stream)
    e = c.energies()
    dt = time.perf_counter() - t0
    kernel_s = ev0.elapsed_time(ev1) / 1e3
    sw1, rot1 = c.work()
    flops = chain_bench.itebd_flops(chi, batch * nup, sw1 - sw0, rot1 - rot0)
    launches = -(-nup // 32)          # itebd_evolve launches up to 32 updates at a time
    out["d30_batch512"] = {"chains": batch, "bond_updates_per_chain": nup, "seconds": dt,
                           "updates_per_s": batch * nup / dt, "us_per_update_per_chain": dt / nup * 1e6,
                           "energy_mean": float(np.mean(e)), "energy_minus_bethe_max": float(np.max(e) - bethe),
                           "energy_minus_bethe_min": float(np.min(e) - bethe),
                           "mean_jacobi_sweeps": (sw1 - sw0) / (batch * nup),
                           "flops_per_update": flops / (batch * nup)}
    # FP64 vector FMAs out of LDS: priced against the FP64 vector peak
    out["roofline"] = {"kernel": "itebd_update_kernel", "bound": "alu", "achieved": flops / kernel_s / 1e12,
                       "peak": 78.6, "unit": "TFLOP/s", "frac": flops / kernel_s / 1e12 / 78.6,
                       "launches": launches, "avg_launch_ms": kernel_s / launches * 1e3,
                       "measured": "HIP events on the chains' stream around 10,000 updates of 512 chains "
                                   "(launches of 32 updates each), FLOPs from the device-side sweep and "
                                   "rotation counters"}
    c.close()
    scan = {}
    for b in (1, 512):
        rows = []
        for d in (4, 8, 12, 16, 20, 24, 30):
            c = binding.Chains(h, workloads.random_chain_states(b, d, seed=d), d)
            c.evolve(0.05, 64)
            c.energies()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.evolve(0.05, 1000)
            c.energies()
            dt = time.perf_counter() - t0
            rows.append((d, dt / 1000 * 1e6))
            c.close()
        x = np.polyfit(np.log([r[0] for r in rows]), np.log([r[1] for r in rows]), 1)[0]
        scan[f"batch{b}"] = {"us_per_update": {str(d): t for d, t in rows}, "fit_exponent": float(x)}
    out["scaling"] = scan
    return out


def run_qchain(binding, workloads, stepping="engine"):
    """HOTRG of the S = 1/2 antiferromagnetic Heisenberg chain mapped onto an
    imaginary-time network (the paper's HOTRG workload), FP64: time per
    coarse-graining step against D_b (12 steps along imaginary time,
    beta = 1, tau = 2^-12) with the fitted exponent of time ~ D_b^x, and the
    free energy per site at several temperatures (D_b = 32)."""
    import math
    import numpy as np
    import torch
    h = workloads.heisenberg_bond()
    out = {"workload": "S=1/2 AF Heisenberg chain, Trotter step tau = beta / 2^k, k steps along imaginary "
                       "time, then the infinite chain (dominant eigenvalue of the column transfer matrix), FP64"}
    k = 12
    tau = 1.0 / 2 ** k
    rows, rows_whole = [], []
    for d in (4, 8, 16, 24, 32, 48):
        s = binding.Solve(model="qchain", bond_h=h, tau=tau, dmax=d, max_steps=k)
        s.coarse_grain(k, exchange=False)
        s.log_z_chain()
        for mode, dest in ((stepping, rows), ("whole", rows_whole)):
            s.reset(model="qchain", bond_h=h, tau=tau, dmax=d, max_steps=k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "engine":
                s.coarse_grain_async(k, exchange=False)    # host-polled steps, the library's thread
            else:
                s.coarse_grain(k, exchange=False)
            s.log_z_chain()
            dest.append((d, (time.perf_counter() - t0) / k * 1e3))
        s.close()
    x = np.polyfit(np.log([r[0] for r in rows[1:]]), np.log([r[1] for r in rows[1:]]), 1)[0]
    out["stepping"] = stepping
    out["ms_per_step"] = {str(d): t for d, t in rows}
    out["ms_per_step_whole_steps"] = {str(d): t for d, t in rows_whole}
    out["fit_exponent_d8_to_d48"] = float(x)
    # where a step goes at D_b = 32: HIP events between the stages of every
    # step (a separate timed solve, so the timing above is not perturbed)
    s = binding.Solve(model="qchain", bond_h=h, tau=tau, dmax=32, max_steps=k)
    s.set_timing(True)
    s.coarse_grain(k, exchange=False)
    s.log_z_chain()
    st, nst = s.stage_times()
    s.close()
    out["stage_ms_per_step_d32"] = {name: v / max(nst, 1) for name, v in st.items() if v > 0.0}
    fe = {}
    for temp in (2.0, 1.0, 0.5, 0.25):
        tau_t = (1.0 / temp) / 2 ** k
        s = binding.Solve(model="qchain", bond_h=h, tau=tau_t, dmax=32, max_steps=k)
        s.coarse_grain(k, exchange=False)
        fe[str(temp)] = -s.log_z_chain() / (2.0 * tau_t)
        s.close()
    s = binding.Solve(model="qchain", bond_h=h, tau=0.05, dmax=32, max_steps=14)
    s.coarse_grain(14, exchange=False)
    e_low = -s.log_z_chain() / 0.1
    s.close()
    out["free_energy_d32"] = fe
    out["beta_819_d32"] = {"free_energy": e_low, "minus_bethe": e_low - (0.25 - math.log(2.0))}
    return out


def run_c5(binding, accounting):
    """Ising at Tc, D = 64, 40 steps, one solve in FP16X3, one in BF16x6 and
    one in FP64 on the same GPU: throughput and |delta f| between them and
    against Onsager."""
    import torch
    ref = onsager_reference()
    tc = ref["critical"]["temperature"] if ref else 2.269185314213022
    flops = accounting.solve_flops(2, 64, 40)
    out = {"workload": "Ising J=1 at Tc, D=64, 40 steps, one solve per precision"}
    lnz = {}
    for prec in ("fp16x3", "bf16x6", "fp64"):
        s = binding.Solve(model="ising", q=2, temperature=tc, dmax=64, precision=prec, max_steps=40)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.coarse_grain(40)
        lnz[prec] = s.log_z()
        dt = time.perf_counter() - t0
        s.close()
        out[prec] = {"seconds": dt, "tflops": flops / dt / 1e12, "lnz_per_site": lnz[prec]}
        if ref:
            out[prec]["rel_df_vs_onsager"] = abs(lnz[prec] - ref["critical"]["lnz_per_site"]) / \
                ref["critical"]["lnz_per_site"]
        del s
        torch.cuda.empty_cache()
    for prec in ("fp16x3", "bf16x6"):
        out[f"rel_df_{prec}_vs_fp64"] = abs(lnz[prec] - lnz["fp64"]) / abs(lnz["fp64"])
        out[f"speedup_{prec}_vs_fp64"] = out["fp64"]["seconds"] / out[prec]["seconds"]
    return out


def cpu_baseline_chains():
    """The oracle on the host for the two chain workloads: iTEBD bond updates
    of one Heisenberg chain at D_b = 30 (400 updates) and quantum-chain HOTRG
    steps along imaginary time at D_b = 16 and 32 (12 steps each)."""
    import numpy as np
    from oracle import itebd as oi, qchain as oq, hotrg as oh
    from paper_2602_05900_amd import workloads as wl
    h = wl.heisenberg_bond()
    st = oi.unpack(wl.random_chain_states(1, 30, seed=2026)[0], 30)
    st = oi.evolve(st, h, 0.1, 20, 30)
    t0 = time.perf_counter()
    oi.evolve(st, h, 0.01, 400, 30)
    it = (time.perf_counter() - t0) / 400
    q = {}
    for d in (16, 32):
        T0 = oq.block_tensor(h, 1.0 / 2 ** 12)
        t0 = time.perf_counter()
        oh.solve_tensor(T0, d, 12, keep_tensor=False, schedule=[False] * 12)
        q[str(d)] = (time.perf_counter() - t0) / 12 * 1e3
    return {"itebd_us_per_update_d30_one_chain": it * 1e6, "itebd_updates_per_s": 1.0 / it,
            "qchain_ms_per_step": q}


def cpu_baseline(dmax: int, nsteps_sample: int, temperature: float):
    """The FP64 oracle, as it stands, on the first steps of one solve of the
    same workload (steps 1..nsteps_sample; the last is a full D^7 step)."""
    from oracle import hotrg as oracle
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads") or 0) for i in threadpool_info()) or None
    except Exception:
        pass
    t0 = time.perf_counter()
    oracle.solve("ising", 2, temperature, dmax, nsteps_sample, keep_tensor=False)
    dt = time.perf_counter() - t0
    flops = sum(oracle.contraction_flops(*d) for d in oracle.step_dims(2, 2, dmax, nsteps_sample))
    return {
        "value": flops / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": threads or os.cpu_count(),
        "kind": "oracle",
        "sample": f"first {nsteps_sample} of 30 steps of one D={dmax} Ising solve at T={temperature:.4f} "
                  f"({flops:.3e} contraction FLOPs in {dt:.2f} s, FP64 NumPy/LAPACK)",
        "seconds": dt,
    }


def run_roofline(binding, accounting, precision, dmax, nsteps, temperature):
    """The dominant kernel, the Y product at steady state (dims D x D x D,
    2 D^7 algorithmic FLOPs a launch), measured alone: one solve on its own
    stream with HIP events around every Y launch, averaged over the
    steady-state launches only (the early, growing steps use other tiles)."""
    s = binding.Solve(model="ising", q=2, temperature=temperature, dmax=dmax, precision=precision,
                      max_steps=nsteps)
    s.set_timing(True)
    s.coarse_grain(nsteps)
    s.log_z()
    per_step = s.step_stage_times()
    s.close()
    steady = [ms["y"] for dims, ms in per_step if dims == (dmax, dmax, dmax)]
    if not steady:
        return {"error": "no steady-state Y launch in this configuration"}
    avg = sum(steady) / len(steady)
    flops = accounting.stage_flops(dmax, dmax, dmax)["y"]
    achieved = flops / (avg * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    traffic = measured_traffic(precision, dmax, nsteps)
    return {
        "kernel": "gemm_nt Y = X . T (the D^7 product), steady-state launch",
        "bound": "mfma",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": traffic,
        "traffic_unit": "HBM bytes per steady launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "algorithmic_flops_per_launch": flops,
        "algorithmic_bytes_per_launch": accounting.y_bytes(dmax, dmax, dmax, ELEM_BYTES[precision],
                                                           Y_OUT_BYTES[precision]),
        "issued_mfma_products": PRODUCTS[precision],
        "issued_achieved": achieved * PRODUCTS[precision],
        "issued_frac": achieved * PRODUCTS[precision] / peak,
        "launches": len(steady),
        "avg_launch_ms": avg,
        "min_launch_ms": min(steady),
        "max_launch_ms": max(steady),
        "measured": "HIP events on the solve's stream around each steady-state Y launch of one solve run alone",
    }


def run_c4(serve, accounting, workloads, precision, slots, budget, stepping="whole"):
    """Served solves under Poisson arrivals (the serving workload's request
    mix), time-bounded: a rate below the knee and the overloaded 50 req/s.
    Requests without a result when the horizon ends are counted and enter
    the latency percentiles with the time they had waited by then (so those
    percentiles are lower bounds under overload)."""
    srv = serve.Server(slots=slots, budget=budget, precision=precision, stepping=stepping)
    out = {"workload": "Poisson arrivals; Ising/Potts(q=3) uniform, T ~ U[0.5, 1.5] Tc, D in {16,24,32,48}, "
                       "20-40 steps, seeded; served with continuous batching",
           "precision": precision, "slots": slots, "stepping": stepping, "runs": []}
    for rate, seconds, horizon in ((10.0, 15.0, 30.0), (50.0, 10.0, 20.0)):
        reqs = workloads.request_stream(rate_hz=rate, duration_s=seconds)
        offered = sum(accounting.solve_flops(r.q, r.dmax, r.nsteps) for r in reqs) / seconds / 1e12

        def progress(now, done, total, active, queued, rate=rate):
            print(f"# C4 {rate:g} req/s {now:6.1f} s: {done}/{total} done, {active} active, {queued} queued",
                  file=sys.stderr, flush=True)

        t0 = time.perf_counter()
        done = srv.run(reqs, realtime=True, progress=progress, horizon=horizon)
        wall = time.perf_counter() - t0
        lat = [c.latency for c in done]
        waited = lat + [max(horizon - a, 0.0) for _, a in srv.unfinished]
        service = [c.finished - c.admitted for c in done]
        out["runs"].append({
            "rate_hz": rate, "arrival_window_s": seconds, "horizon_s": horizon, "requests": len(reqs),
            "finished": len(done), "unfinished": len(srv.unfinished), "wall_s": wall,
            "offered_tflops": offered,
            "served_tflops": sum(c.flops for c in done) / wall / 1e12,
            "solves_per_s": len(done) / wall,
            "p50_latency_s": serve.percentile(lat, 50), "p99_latency_s": serve.percentile(lat, 99),
            "p50_latency_s_all_requests_lower_bound": serve.percentile(waited, 50),
            "p99_latency_s_all_requests_lower_bound": serve.percentile(waited, 99),
            "p50_service_s": serve.percentile(service, 50), "p99_service_s": serve.percentile(service, 99),
            "peak_footprint_gb": srv.peak_in_use / 2 ** 30,
        })
        srv.peak_in_use = srv.in_use
    return out


def run_leg(line, name, fn, *args):
    """One side measurement: its result, or its error, under its own key, so
    that a failing leg never drops the benchmark line."""
    print(f"# {name} ...", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    try:
        line[name] = fn(*args)
    except Exception as e:  # noqa: BLE001 - recorded in the line
        traceback.print_exc(file=sys.stderr)
        line[name] = {"error": f"{type(e).__name__}: {e}"}
    if isinstance(line[name], dict):
        line[name]["leg_wall_s"] = time.perf_counter() - t0


def finite(obj):
    """The line with every non-finite float replaced by null (strict JSON)."""
    if isinstance(obj, float):
        return obj if math.isfinite(obj) else None
    if isinstance(obj, dict):
        return {k: finite(v) for k, v in obj.items()}
    if isinstance(obj, (list, tuple)):
        return [finite(v) for v in obj]
    return obj


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves")
    ap.add_argument("--precision", default="fp16x3", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--no-compare-fp64", dest="compare_fp64", action="store_false",
                    help="skip the FP64 run of the same batch")
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="skip the BF16x6, FP32 and FP64 runs of the same batch")
    ap.add_argument("--dmax", type=int, default=48)
    ap.add_argument("--nsteps", type=int, default=30, help="coarse-graining steps per solve")
    ap.add_argument("--cpu-sample-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--concurrency", type=int, default=4, help="solves in flight (streams)")
    ap.add_argument("--stepping", default="whole", choices=["whole", "polled", "engine", "hybrid"],
                    help="whole steps (every eigensolver pass up to the cap enqueued), host-polled steps "
                         "driven by the scheduler, or by the library's progress thread")
    ap.add_argument("--latency-stepping", default="engine", choices=["whole", "engine"],
                    help="steps of the one-solve-at-a-time legs (C2 scan, observables, quantum chain): whole steps or "
                         "host-polled steps driven by the library's progress thread")
    ap.add_argument("--budget-gb", type=int, default=128, help="device memory for solve workspaces")
    ap.add_argument("--no-c2", dest="c2", action="store_false", help="skip the D=24 temperature scan")
    ap.add_argument("--no-c4", dest="c4", action="store_false", help="skip the served Poisson stream")
    ap.add_argument("--no-c5", dest="c5", action="store_false", help="skip the D=64 solve")
    ap.add_argument("--no-observables", dest="observables", action="store_false",
                    help="skip the two-sided / impurity-observable runs")
    ap.add_argument("--no-itebd", dest="itebd", action="store_false", help="skip the iTEBD runs")
    ap.add_argument("--no-qchain", dest="qchain", action="store_false", help="skip the quantum-chain HOTRG runs")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: the path has no multi-GPU mode, so --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2602_05900_amd import accounting, binding, serve, workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    temps = workloads.temperature_grid(2.0, 2.5, 16)
    flops_solve = accounting.solve_flops(2, args.dmax, args.nsteps)

    def batch(first, count):
        return [workloads.Request(rid=first + i, arrival=0.0, model="ising", q=2,
                                  temperature=float(temps[(first + i) % len(temps)]), dmax=args.dmax,
                                  nsteps=args.nsteps) for i in range(count)]

    def progress(now, done, total, active, queued):
        print(f"# {now:6.1f} s: {done}/{total} solves done, {active} active", file=sys.stderr, flush=True)

    def run_batch(precision, concurrency, warm_reqs, reqs):
        server = serve.Server(slots=concurrency, budget=args.budget_gb << 30, precision=precision,
                              device="cuda:0", timing=True, stepping=args.stepping)
        if warm_reqs:
            server.run(warm_reqs, realtime=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = server.run(reqs, realtime=False, progress=progress)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stage = {k: 0.0 for k in binding.STAGES}
        for c in done:
            for k, v in (c.stage_ms or {}).items():
                stage[k] += v
        print(f"# {precision}: {len(reqs)} solves, {concurrency} in flight, {wall:.2f} s", file=sys.stderr,
              flush=True)
        return done, wall, stage

    # the timed batch: solves warmup .. warmup + steps - 1 of the temperature cycle
    warm_reqs, timed_reqs = batch(0, args.warmup), batch(args.warmup, args.steps)
    done, wall, stage_sum = run_batch(args.precision, args.concurrency, warm_reqs, timed_reqs)
    for c in done:
        print(f"# solve T={c.temperature:.4f} lnZ/N={c.lnz_per_site:.15f} service "
              f"{1e3 * (c.finished - c.admitted):.1f} ms", file=sys.stderr, flush=True)

    total_flops = flops_solve * args.steps
    value = total_flops / wall / 1e12
    contraction_ms = stage_sum["env"] + stage_sum["x"] + stage_sum["y"] + stage_sum["tp"]
    service = [c.finished - c.admitted for c in done]
    latency = [c.latency for c in done]

    ref = {}
    ref_path = os.path.join(ROOT, "tests", "golden", "oracle_ising_d48.json")
    if args.dmax == 48 and args.nsteps == 30 and os.path.exists(ref_path):
        ref = {round(r["temperature"], 9): r["lnz_per_site"] for r in json.load(open(ref_path))["rows"]}
    errs = {}
    for c in done:
        key = round(c.temperature, 9)
        if key in ref:
            errs[f"{c.temperature:.6f}"] = abs(c.lnz_per_site - ref[key]) / abs(ref[key])

    line = {
        "metric": "HOTRG contraction TFLOP/s at D=48 (FP64 vs mixed); p50/p99 solve latency",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"HOTRG 2D Ising J=1, D={args.dmax}, {args.nsteps} steps per solve, "
                        f"T cycling over 16 values in [2.0, 2.5]; one step of this benchmark = one solve; "
                        f"{args.concurrency} solves in flight on separate streams",
            "dmax": args.dmax,
            "coarse_grain_steps": args.nsteps,
            "contraction_precision": args.precision,
            "eigensolve": "FP64",
            "concurrency": args.concurrency,
            "stepping": args.stepping,
            "latency_stepping": args.latency_stepping,
            "flops_per_solve": flops_solve,
        },
        "p50_solve_ms": serve.percentile(service, 50) * 1e3,
        "p99_solve_ms": serve.percentile(service, 99) * 1e3,
        "p50_batch_latency_ms": serve.percentile(latency, 50) * 1e3,
        "p99_batch_latency_ms": serve.percentile(latency, 99) * 1e3,
        "solves_per_s": args.steps / wall,
        "stage_ms_per_solve": {k: v / args.steps for k, v in stage_sum.items()},
        "contraction_kernel_tflops": total_flops / (contraction_ms * 1e-3) / 1e12 if contraction_ms else None,
        "lnz_per_site": {f"{c.temperature:.6f}": c.lnz_per_site for c in done},
        "rel_err_vs_fp64_oracle": errs or None,
        "max_rel_err_vs_fp64_oracle": max(errs.values()) if errs else None,
    }
    run_leg(line, "roofline", run_roofline, binding, accounting, args.precision, args.dmax, args.nsteps,
            float(temps[0]))

    def comparison(prec):
        # the same requests (same temperatures) as the timed batch, one warm-up solve first
        fdone, fwall, _ = run_batch(prec, args.concurrency, batch(0, 1), timed_reqs)
        fl = {c.rid: c.lnz_per_site for c in fdone}
        out = {
            "precision": prec,
            "value": flops_solve * args.steps / fwall / 1e12,
            "ms_per_step": fwall / args.steps * 1e3,
            "headline_speedup": fwall / wall,
            "max_rel_df_headline_vs_this": max(abs(c.lnz_per_site - fl[c.rid]) / abs(fl[c.rid]) for c in done),
        }
        ferr = [abs(c.lnz_per_site - ref[round(c.temperature, 9)]) / abs(ref[round(c.temperature, 9)])
                for c in fdone if round(c.temperature, 9) in ref]
        if ferr:
            out["max_rel_err_vs_fp64_oracle"] = max(ferr)
        return out

    # the same requests in the other precisions of the mixed-precision
    # workload (FP32 and BF16 split contractions) and in FP64
    for prec in ("bf16x6", "fp32", "fp64"):
        if prec != args.precision and args.compare and (prec != "fp64" or args.compare_fp64):
            run_leg(line, f"{prec}_comparison", comparison, prec)
    if args.c2:
        run_leg(line, "c2", run_c2, serve, accounting, workloads, args.budget_gb << 30, args.latency_stepping)
    if args.c4:
        run_leg(line, "c4", run_c4, serve, accounting, workloads, args.precision, 8, 160 << 30,
                args.stepping)
    if args.c5:
        run_leg(line, "c5", run_c5, binding, accounting)
    if args.observables:
        run_leg(line, "observables", run_observables, binding, accounting, args.latency_stepping)
    if args.itebd:
        run_leg(line, "itebd", run_itebd, binding, workloads)
    if args.qchain:
        run_leg(line, "qchain", run_qchain, binding, workloads, args.latency_stepping)
    if not args.no_cpu_baseline:
        def cpu():
            out = cpu_baseline(args.dmax, args.cpu_sample_steps, float(temps[0]))
            out["chains"] = cpu_baseline_chains()
            return out
        run_leg(line, "cpu_baseline", cpu)
    print(json.dumps(finite(line)), flush=True)


if __name__ == "__main__":
    main()

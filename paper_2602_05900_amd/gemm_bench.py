"""Run the contraction kernel alone on the shape of one HOTRG product.

    python -m paper_2602_05900_amd.gemm_bench [--role y] [--dmax 48] [--precision fp16x3] [--reps 5]
                                              [--copy-mib 1024]

Shapes at steady state (Dx = Dy = D' = D): y: M = D^3, N = K = D^2 (the D^7
term); x: M = D^2, N = D^3, K = D; tp: M = D^3, N = D, K = D^2; env: M = N =
K = D^2.  Operands are random FP64 device tensors.  For the reduced
precisions hotrg_gemm_nt_role first splits them into BF16 or FP16 planes (or
rounds them to FP32) with a conversion kernel and then runs the kernel a
solve launches for that role (the split operands of the y and env roles in
the panel layout, as a solve's producers write them); the time printed
covers both launches, so it is an upper bound on the product kernel's own
duration (a kernel trace separates the two).

--copy-mib S first copies S MiB between two device buffers with a plain
device-to-device copy, so that a hardware-counter run of this module also
records a kernel of known traffic (S MiB read, S MiB written) for scaling
the counters.  One JSON line per run.
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--role", default="y", choices=["y", "x", "tp", "env"])
    ap.add_argument("--dmax", type=int, default=48)
    ap.add_argument("--precision", default="fp16x3")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=0)
    args = ap.parse_args()
    import torch
    from . import binding
    D = args.dmax
    M, N, K = {"y": (D ** 3, D ** 2, D ** 2), "x": (D ** 2, D ** 3, D), "tp": (D ** 3, D, D ** 2),
               "env": (D ** 2, D ** 2, D ** 2)}[args.role]
    copy = None
    if args.copy_mib > 0:
        n = args.copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        copy = {"bytes": n}
        del src, dst
    A = torch.randn(M, K, dtype=torch.float64, device="cuda")
    B = torch.randn(N, K, dtype=torch.float64, device="cuda")
    C = torch.empty(M * N, dtype=torch.float64, device="cuda")
    split = args.precision in ("bf16x3", "bf16x6", "fp16x3")
    kw = dict(precision=args.precision, role={"env": "generic"}.get(args.role, args.role),
              panel=split and args.role in ("y", "env"))
    binding.gemm_nt(A, B, C, M, N, K, K, K, (1, N, 0, 1, 1, 0), **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.reps):
        binding.gemm_nt(A, B, C, M, N, K, K, K, (1, N, 0, 1, 1, 0), **kw)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.reps
    flops = 2.0 * M * N * K
    print(json.dumps({"role": args.role, "dmax": D, "M": M, "N": N, "K": K, "precision": args.precision,
                      "ms_per_call_incl_conversion": ms, "algorithmic_tflops": flops / ms / 1e9,
                      "calibration_copy": copy}), flush=True)


if __name__ == "__main__":
    main()

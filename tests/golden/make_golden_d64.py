"""Writes tests/golden/oracle_ising_d64.json: the FP64 oracle's run of the 2D
Ising model at the critical temperature with bond dimension D = 64 for the
first 10 coarse-graining steps (environments of n = 4096 from step 7 on):
ln Z/N of the 2^10-site torus, every normalisation c_n, truncation error and
gap at the cut.  Calls oracle/ only.

    python tests/golden/make_golden_d64.py      (several CPU-minutes, ~30 GB of memory)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact, hotrg  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "oracle_ising_d64.json")
NSTEPS = 10


def main():
    T = exact.ISING_TC
    t0 = time.time()
    s = hotrg.solve("ising", 2, T, 64, NSTEPS, keep_tensor=False)
    out = {"about": f"FP64 oracle (oracle/hotrg.py), Ising J=1 at Tc, D=64, the first {NSTEPS} steps",
           "temperature": T, "dmax": 64, "nsteps": NSTEPS, "lnz_per_site": s.lnz_per_site,
           "c": s.c, "trunc_err": s.trunc_err, "cut_gap": [g if g != float("inf") else None for g in s.cut_gap],
           "dims": s.dims, "seconds": time.time() - t0}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"lnZ/N={s.lnz_per_site:.16f} ({time.time() - t0:.1f} s)")


if __name__ == "__main__":
    main()

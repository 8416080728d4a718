"""Writes tests/golden/oracle_ising_d32.json: the FP64 oracle's ln Z/N for the
2D Ising model at D = 32 after 30 steps at T = 2.0, Tc and 2.5 (the smallest
bond dimension whose steady-state Y product runs on the full-size tiles).
Calls oracle/ only.

    python tests/golden/make_golden_d32.py      (about a minute per temperature on 8 cores)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact, hotrg  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "oracle_ising_d32.json")


def main():
    rows = []
    for T in (2.0, exact.ISING_TC, 2.5):
        t0 = time.time()
        s = hotrg.solve("ising", 2, float(T), 32, 30, keep_tensor=False)
        rows.append({"temperature": float(T), "lnz_per_site": s.lnz_per_site,
                     "free_energy": -float(T) * s.lnz_per_site, "seconds": time.time() - t0})
        print(f"T={T:.6f} lnZ/N={s.lnz_per_site:.16f} ({time.time() - t0:.1f} s)", flush=True)
    with open(OUT, "w") as f:
        json.dump({"about": "FP64 oracle (oracle/hotrg.py), Ising J=1, D=32, 30 steps, T = 2.0, Tc, 2.5",
                   "rows": rows}, f, indent=1)


if __name__ == "__main__":
    main()

"""Writes tests/golden/oracle_ising_d48.json: the FP64 oracle's ln Z/N for the
2D Ising model at D = 48 after 30 steps, at the 16 temperatures of the
benchmark (numpy.linspace(2.0, 2.5, 16)).  Calls oracle/ only.

    python tests/golden/make_golden_d48.py      (about 5 min per temperature on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import hotrg  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "oracle_ising_d48.json")


def main():
    temps = np.linspace(2.0, 2.5, 16)
    rows = []
    for T in temps:
        t0 = time.time()
        s = hotrg.solve("ising", 2, float(T), 48, 30, keep_tensor=False)
        rows.append({"temperature": float(T), "lnz_per_site": s.lnz_per_site,
                     "free_energy": -float(T) * s.lnz_per_site, "seconds": time.time() - t0})
        print(f"T={T:.6f} lnZ/N={s.lnz_per_site:.16f} ({time.time() - t0:.1f} s)", flush=True)
        with open(OUT, "w") as f:
            json.dump({"about": "FP64 oracle (oracle/hotrg.py), Ising J=1, D=48, 30 steps, "
                                "T = numpy.linspace(2.0, 2.5, 16)", "rows": rows}, f, indent=1)


if __name__ == "__main__":
    main()

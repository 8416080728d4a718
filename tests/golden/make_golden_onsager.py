"""Writes tests/golden/onsager_ising.json: Onsager's exact ln Z/N and internal
energy per site of the infinite 2D Ising model (J = 1) on the temperature
grid of the D = 24 scan (numpy.linspace(1.8, 2.8, 64)) and at the critical
point, the spontaneous magnetisation (Yang) on that grid, plus the
central-difference energy of the exact ln Z/N on that grid (the
discretisation error any finite-difference energy on it carries).
Calls oracle/ only.

    python tests/golden/make_golden_onsager.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "onsager_ising.json")


def main():
    temps = np.linspace(1.8, 2.8, 64)
    lnz = np.array([exact.onsager_lnz(float(t)) for t in temps])
    u = np.array([exact.onsager_energy(float(t)) for t in temps])
    u_fd = exact.finite_difference_energy(temps, lnz)
    tc = exact.ISING_TC
    out = {
        "about": "Onsager's exact solution (oracle/exact.py), 2D Ising J=1; grid = numpy.linspace(1.8, 2.8, 64)",
        "grid": {"temperatures": temps.tolist(), "lnz_per_site": lnz.tolist(), "energy": u.tolist(),
                 "energy_fd_of_exact_lnz": u_fd.tolist(),
                 "magnetisation": [exact.yang_magnetisation(float(t)) for t in temps]},
        "critical": {"temperature": tc, "lnz_per_site": exact.onsager_lnz_tc(),
                     "energy": exact.onsager_energy(tc)},
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(OUT)


if __name__ == "__main__":
    main()

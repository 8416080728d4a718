"""Writes tests/golden/exact_tori.json from the independent routes in
oracle/exact.py only (brute-force spin sums and the spin transfer matrix).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402


def main():
    cases = []
    ising_temps = [1.5, exact.ISING_TC, 3.0]
    potts_temps = [0.7, exact.POTTS3_TC, 1.4]
    for nsteps in range(0, 5):
        Lx, Ly = exact.hotrg_torus(nsteps)
        for T in ising_temps:
            lnz = exact.brute_force_lnz("ising", 2, T, Lx, Ly)
            cases.append({"model": "ising", "q": 2, "temperature": T, "nsteps": nsteps,
                          "Lx": Lx, "Ly": Ly, "lnz_per_site": lnz / (Lx * Ly),
                          "route": "brute force over 2^(Lx*Ly) states"})
        for T in potts_temps:
            if 3 ** (Lx * Ly) <= 6561:
                lnz = exact.brute_force_lnz("potts", 3, T, Lx, Ly)
                route = "brute force over 3^(Lx*Ly) states"
            else:
                lnz = exact.spin_transfer_lnz("potts", 3, T, Lx, Ly)
                route = "row transfer matrix over 3^Lx row states"
            cases.append({"model": "potts", "q": 3, "temperature": T, "nsteps": nsteps,
                          "Lx": Lx, "Ly": Ly, "lnz_per_site": lnz / (Lx * Ly), "route": route})
    doc = {
        "about": ("ln Z / N of small periodic tori of the square-lattice Ising (J=1) and "
                  "3-state Potts (J=1) models, Z = Tr exp(-beta H) (Sec. II.A); the torus "
                  "for n HOTRG steps is 2^floor(n/2) x 2^ceil(n/2) sites (x by y)."),
        "onsager_tc": {
            "temperature": 2.0 / math.log(1.0 + math.sqrt(2.0)),
            "lnz_per_site": 0.5 * math.log(2.0) + 2.0 * exact.CATALAN / math.pi,
            "source": "Onsager (1944) at the critical point: (1/2) ln 2 + 2G/pi, G = Catalan's constant",
        },
        "cases": cases,
    }
    path = os.path.join(ROOT, "tests", "golden", "exact_tori.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {len(cases)} cases to {path}")


if __name__ == "__main__":
    main()

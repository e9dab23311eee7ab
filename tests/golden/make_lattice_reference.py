"""Write tests/golden/lattice_reference.json: exact <E>/N and <m> of general
lattices by the row transfer matrix of oracle.exact (oracle only).

  * the laterally confined strip of Sec. III.A (Fig. 3f): 12 columns open,
    18 rows periodic, J2/J1 = 1.5, h/J1 = 4.5, at T = 1.0, 0.7, 0.5, 0.3;
  * the same strip at h/J1 = 2.5 and 3.5 (at and below the confined
    transition), T = 1.0, 0.7, 0.5;
  * a 12 x 12 periodic lattice with different fields on even and odd columns
    (App. A Accumulator), J2/J1 = 1, h_even = 3.5, h_odd = 2.5, T = 0.8;
  * a lattice with ten different filter couplings (App. A Convoluter-Reverse),
    8 columns open, 12 rows periodic, T = 0.8.

Run from the repository root:  python tests/golden/make_lattice_reference.py
"""
from __future__ import annotations

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lattice_reference.json")

SS = lambda J1, J2: [J1] * 8 + [J2] * 2  # noqa: E731
RAW_J = [1.0, 0.8, -0.6, 1.2, 0.9, -1.1, 0.5, 1.4, 1.3, -0.7]


def main():
    cases = []
    for h, temps in ((4.5, (1.0, 0.7, 0.5, 0.3)), (3.5, (1.0, 0.7, 0.5)), (2.5, (1.0, 0.7, 0.5))):
        for T in temps:
            cases.append({"name": f"strip12x18_h{h}_T{T}", "rows": 18, "cols": 12, "open_rows": False,
                          "open_cols": True, "J": SS(1.0, 1.5), "h_even": h, "h_odd": h, "T": T,
                          "cite": "Sec. III.A, Fig. 3f: SS lattice of 12 x 18 with lateral confinement, "
                                  "J2/J1 = 1.5"})
    cases.append({"name": "periodic12_oddeven_T0.8", "rows": 12, "cols": 12, "open_rows": False,
                  "open_cols": False, "J": SS(1.0, 1.0), "h_even": 3.5, "h_odd": 2.5, "T": 0.8,
                  "cite": "App. A Accumulator: separate even and odd column biases"})
    cases.append({"name": "raw_filters_8x12_T0.8", "rows": 12, "cols": 8, "open_rows": False, "open_cols": True,
                  "J": RAW_J, "h_even": 0.4, "h_odd": 0.4, "T": 0.8,
                  "cite": "App. A Convoluter-Reverse: every filter written by the host"})
    for c in cases:
        r = exact.lattice_tm_averages(c["rows"], c["cols"], c["J"], c["h_even"], c["h_odd"], c["T"],
                                      open_r=c["open_rows"], open_c=c["open_cols"])
        c["E_per_spin"], c["m"] = r["E"], r["m"]
        print(c["name"], r, flush=True)
    with open(OUT, "w") as f:
        json.dump({"_about": "exact <E>/N and <m> by the row transfer matrix of oracle.exact; written by "
                             "tests/golden/make_lattice_reference.py", "cases": cases}, f, indent=1)


if __name__ == "__main__":
    main()

"""Writes plateau_reference.json: exact <E>/N and <m> of the SS Ising law at
the paper's 1/3-plateau point (J1, J2, h) = (1, 1, 3) (Sec. III.A, Fig. 3e)
for T in {0.1, 0.2, 0.4}, from the row transfer matrix of oracle.exact on the
periodic 6x6 and 12x12 lattices.  The two sizes agree to 1e-14 at T <= 0.2
and to 5e-7 at T = 0.4, so finite-size corrections in this gapped phase are
negligible and the 12x12 values serve as the reference for 18x18 runs.
Calls only oracle/.

    python tests/golden/make_plateau_reference.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
from oracle import exact  # noqa: E402

J1, J2, H = 1.0, 1.0, 3.0
out = {"_about": "Exact <E>/N and <m> at the 1/3-plateau point by row transfer matrix; "
                 "written by make_plateau_reference.py (oracle.exact only).",
       "point": {"J1": J1, "J2": J2, "h": H, "cite": "Sec. III.A (1/3 plateau at J2/J1 = 1.0, hz = 3.0)"},
       "values": []}
for T in (0.1, 0.2, 0.4):
    for L in (6, 12):
        r = exact.tm_averages(L, J1, J2, H, T)
        out["values"].append({"L": L, "T": T, "E_per_spin": r["E"], "m": r["m"]})
        print(L, T, r, flush=True)
path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plateau_reference.json")
with open(path, "w") as f:
    json.dump(out, f, indent=1)

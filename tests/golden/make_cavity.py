"""Writes cavity_ra1e4_oracle.json (or, with the argument 1e6,
cavity_ra1e6_oracle.json): the FP64 oracle's steady natural convection in
the App. D square cavity from rest at the cold temperature, dx = 0.2 mm,
dt = 0.2 ms as in App. D.
  Ra = 1e4: L = 13 mm, 65 x 65 nodes, 40 000 steps (about a minute on one core);
  Ra = 1e6: L = 60 mm, 300 x 300 nodes, 260 000 steps (about 100 minutes).
Stores the mean Nusselt number over the cavity, the hot-wall Nusselt number,
and the mid-height and mid-width profiles of u, v and T.

Calls only the oracle and the seeded workload generator:
  python tests/golden/make_cavity.py [1e4|1e6]"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from paper_2302_04120_amd import workloads as WL  # noqa: E402
from cavity_ref import nusselt_mean, nusselt_hot_wall  # noqa: E402

CASES = {1e4: (40_000, 5_000), 1e6: (260_000, 20_000)}  # steps, report interval


def main(Ra):
    STEPS, every = CASES[Ra]
    prm, ini = WL.cavity(Ra)
    n = ini["rho"].shape[0]
    ch = O.Chan(n, n, prm, bc_x="walls_T", bc_y="walls", thermal=True)
    ch.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    prev = None
    for k in range(STEPS // every):
        ch.step(every)
        m = ch.macros()
        nu = nusselt_mean(m["ux"], m["T"], prm)
        print("%d steps: Nu %.6f" % ((k + 1) * every, nu), flush=True)
        last_change = None if prev is None else abs(nu - prev)
        prev = nu
    m = ch.macros()
    mid = n // 2
    out = {"what": "FP64 oracle, App. D cavity, Ra %.0e" % Ra, "n": n, "steps": STEPS,
           "report_every": every,
           "Ra": prm["Ra"], "Nu_mean": nusselt_mean(m["ux"], m["T"], prm),
           "Nu_hot_wall": nusselt_hot_wall(m["T"], prm),
           "Nu_change_last_interval": last_change,
           "row_mid_uy": m["uy"][mid].tolist(), "row_mid_T": m["T"][mid].tolist(),
           "col_mid_ux": m["ux"][:, mid].tolist(), "col_mid_T": m["T"][:, mid].tolist()}
    name = "cavity_ra%s_oracle.json" % ("1e4" if Ra == 1e4 else "1e6")
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=0)
    print("Nu mean %.5f, hot wall %.5f" % (out["Nu_mean"], out["Nu_hot_wall"]))


if __name__ == "__main__":
    main(float(sys.argv[1]) if len(sys.argv) > 1 else 1e4)

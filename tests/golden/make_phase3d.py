"""Writes tests/golden/phase3d_sphere_oracle.json: the FP64 oracle's 3D
two-phase model (Sec. 2.3 on D3Q19) on a gas sphere, R = 10 dx, in a 40^3
periodic box of the C3 air/water-like properties, run to a steady pressure
jump.  Calls only the oracle and the seeded input module.  About 4 minutes.

    python tests/golden/make_phase3d.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2302_04120_amd import workloads as WL  # noqa: E402

N, R_NODES, STEPS, INTERVAL, SEED = 40, 10.0, 2400, 400, 0


def jump(o, prm, centre, R):
    m = o.macros()
    x = WL.node_centres(N, prm["dx"])
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2)
    W = prm["W"]
    dP = m["p"][r < R - 2 * W].mean() - m["p"][r > R + 2 * W].mean()
    rho_a = prm["rho_g"] + WL.tanh_profile(r - R, W) * (prm["rho_l"] - prm["rho_g"])
    return dP, m, O.e2(rho_a, m["rho"])


def main():
    prm, ini = WL.bubble3d(n=N, R_nodes=R_NODES, seed=SEED)
    o = O.Phase3(N, N, N, prm)
    o.init(ini["phi"][0], ini["p"][0], ini["ux"][0], ini["uy"][0], ini["uz"][0])
    x = WL.node_centres(N, prm["dx"])
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    gas = ini["phi"][0] < 0.5
    centre = (X[gas].mean(), Y[gas].mean(), Z[gas].mean())
    R = R_NODES * prm["dx"]
    s0 = float(ini["phi"][0].sum())
    hist = []
    for k in range(STEPS // INTERVAL):
        o.step(INTERVAL)
        dP, m, e2 = jump(o, prm, centre, R)
        hist.append(dP)
        print("%d steps: dP %.3f Pa (2 sigma / R = %.3f)" % ((k + 1) * INTERVAL, dP, 2 * prm["sigma"] / R),
              flush=True)
    out = dict(case="gas sphere R = 10 dx in a 40^3 periodic box, C3 properties, FP64 oracle",
               n=N, R=R, R_nodes=R_NODES, steps=STEPS, seed=SEED, sigma=prm["sigma"],
               dx=prm["dx"], dt=prm["dt"], W=prm["W"], dP=hist[-1],
               dP_change_last_interval=hist[-1] - hist[-2], dP_history=hist,
               phi_sum_start=s0, phi_sum_end=float(m["phi"].sum()), rho_e2_percent=e2,
               umax=float(max(np.abs(m[k]).max() for k in ("ux", "uy", "uz"))))
    with open(os.path.join(HERE, "phase3d_sphere_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()

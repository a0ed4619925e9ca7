"""Writes layered_coarse_oracle.json: the FP64 oracle's steady layered
Poiseuille profile on the coarsest grid of the paper's grid study (Sec. 4.4:
dx = 5 um, dt = 0.1 us, W = 25 um = 5 dx), 128 nodes across (H = 0.64 mm),
4 nodes along x, run for 3e6 steps (0.3 s, about 6.5 times the slowest
decay time 4 h^2 / (pi^2 nu_l) = 0.046 s of the liquid layer).

Calls only the oracle and the seeded workload generator.  Takes about
15 minutes on one core:  python tests/golden/make_layered_coarse.py"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from paper_2302_04120_amd import workloads as WL  # noqa: E402
from layered_ref import diffuse_profile, sharp_profile  # noqa: E402

NY, DX, DT, STEPS = 128, 5e-6, 1e-7, 3_000_000


def case():
    return WL.layered(nx=4, ny=NY, seed=0, dx=DX, dt=DT, W_nodes=5.0)


def main():
    prm, ini, offs = case()
    ph = O.Phase(4, NY, prm, bc_y="walls")
    ph.init(ini["phi"][0], ini["p"][0], ini["ux"][0], ini["uy"][0])
    y = WL.node_centres(NY, DX)
    H = NY * DX
    t0 = time.time()
    chunk = 250_000
    prev = None
    change = None
    for k in range(STEPS // chunk):
        ph.step(chunk)
        u = ph.macros()["ux"][:, 0]
        if prev is not None:
            change = float(np.abs(u - prev).max() / np.abs(u).max())
        prev = u
        print("%d steps, max relative change over the last %d: %s (%.0f s)" %
              ((k + 1) * chunk, chunk, change, time.time() - t0), flush=True)
    m = ph.macros()
    u, phi = m["ux"][:, 0], m["phi"][:, 0]
    ud = diffuse_profile(y, phi, prm, H)
    us = sharp_profile(y, offs[0], prm, H)
    out = {"what": "FP64 oracle, layered Poiseuille, coarse grid of the Sec. 4.4 grid study",
           "ny": NY, "nx": 4, "dx": DX, "dt": DT, "W_nodes": 5.0, "seed": 0, "steps": STEPS,
           "last_chunk_max_rel_change": change,
           "E2_vs_diffuse_percent": O.e2(ud, u), "E2_vs_sharp_percent": O.e2(us, u),
           "y_interface": offs[0], "y": y.tolist(), "ux": u.tolist(), "phi": phi.tolist(),
           "uy_max_abs": float(np.abs(m["uy"]).max())}
    with open(os.path.join(HERE, "layered_coarse_oracle.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("E2 vs diffuse %.3f %%, vs sharp %.3f %%" % (out["E2_vs_diffuse_percent"],
                                                     out["E2_vs_sharp_percent"]))


if __name__ == "__main__":
    main()

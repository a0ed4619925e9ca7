"""The layered two-phase channel (Sec. 4.4) at the paper's finest grid run
from rest to steady state: saturated water and steam at 25 C, 4 x 512 nodes
(dx = 1.25 um, dt = 12.5 ns, W = 20 dx, H = 0.64 mm), FP32 storage with FP64
step arithmetic, the many-steps kernel, 6.5 decay times of the liquid
layer's slowest mode (2.42e7 steps, about 100 s).  The steady profile against
the diffuse-interface reference (the steady momentum balance of Eq.
NSE_for_layered_poiseuille integrated with the simulated phi): E2 = 1.28 %
(FP64 gives the same to the printed digits; the paper's table lists 0.817 %
for H = 0.5 mm)."""
import math
import time

import numpy as np
import pytest

from paper_2302_04120_amd import workloads as WL

from gpu_cases import print_case
from layered_ref import diffuse_profile

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_layered_channel_full_grid_steady_state():
    from paper_2302_04120_amd import lbm
    props = {k: v for k, v in WL.TWO_PHASE_SYSTEMS["sat_water_25C"].items()
             if k in ("rho_l", "rho_g", "nu_l", "nu_g", "sigma")}
    ny = 512
    prm, ini, _ = WL.layered(nx=4, ny=ny, seed=0, dx=1.25e-6, dt=1.25e-8, W_nodes=20.0, **props)
    L = lbm.Lattice("phase", 4, ny, prec="fp32_arith64", bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
    L.set_step_fusion(3)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    H = ny * prm["dx"]
    h = 0.5 * H
    steps = int(math.ceil(6.5 * 4 * h * h / (math.pi ** 2 * prm["nu_l"]) / prm["dt"]))
    print_case(test="c4-steady", steps=steps)
    done, chunk, prev = 0, 2_000_000, None
    t0 = time.perf_counter()
    while done < steps:
        n = min(chunk, steps - done)
        if done + n >= steps:
            prev = L.macros(("ux",))["ux"][0, :, 0]
        L.step(n)
        done += n
        print("c4 steady: %d / %d steps, %.1f s" % (done, steps, time.perf_counter() - t0),
              flush=True)
    assert L.first_nonfinite_step() == -1
    m = L.macros(("ux", "phi"))
    L.close()
    u, phi = m["ux"][0, :, 0], m["phi"][0, :, 0]
    y = (np.arange(ny) + 0.5) * prm["dx"]
    ref = diffuse_profile(y, phi, prm, H)
    e2 = 100.0 * np.sqrt(np.sum((ref - u) ** 2) / np.sum(ref ** 2))
    change = float(np.abs(u - prev).max() / np.abs(u).max())
    print("E2 vs diffuse reference %.3f %%, change over the last %d steps %.2e" %
          (e2, n, change), flush=True)
    assert change < 1e-3
    assert e2 == pytest.approx(1.28, abs=0.05)

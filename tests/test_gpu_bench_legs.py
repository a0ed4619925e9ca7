"""The secondary bench legs at their full sizes and launch configurations,
on outputs the oracle can compute:

* C4's layered channel as 4096 replicas of 4 x 512 nodes (FP32, one launch
  per step): sampled replicas against the oracle run one by one;
* the heated channel on 16384 x 2048 nodes (FP32, velocity inlet, pressure
  outlet, flux walls), started from a state that does not vary along x:
  after k steps every node more than k columns from the inlet and the outlet
  has seen only x-invariant data, so it equals the same node of an x-periodic
  channel of the same height, which the oracle runs on 8 columns.  Sampled
  interior columns are compared with it, and all interior columns must
  agree with each other to the bit."""
import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

from gpu_cases import FP32_TOL, density_scale, print_case, rel_err, u_abs_err, u_resolution, u_tol

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_layered_batch_leg_sampled():
    from paper_2302_04120_amd import lbm
    batch, steps = 4096, 20
    prm, ini, _ = WL.layered(nx=4, ny=512, batch=batch, seed=0)
    print_case(test="layered-batch-leg", batch=batch, steps=steps)
    L = lbm.Lattice("phase", 4, 512, batch=batch, prec="fp32", bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    m0 = L.reduce(("phase",))["phase"]
    L.step(steps)
    red = L.reduce(("phase", "nonfinite"))
    assert red["nonfinite"].sum() == 0
    assert (np.abs(red["phase"] - m0) / m0).max() < 1e-13
    g = L.macros(("phi", "p", "ux", "uy"))
    for b in (0, 1234, 4095):
        o = O.Phase(4, 512, prm, bc_y="walls")
        o.init(ini["phi"][b], ini["p"][b], ini["ux"][b], ini["uy"][b])
        o.step(steps)
        mo = o.macros()
        scale_p = max(float(np.abs(mo["p"]).max()), prm["sigma"] / prm["W"])
        # The z_i carry the pressure scale p / c_s^2 while the gas momentum is
        # rho_g u, so FP32 resolves the gas velocity only to EPS32 c (max p /
        # c_s^2) / rho_g (2e-6 m/s here, against |u| ~ 6e-4 m/s after 20
        # steps): gpu_cases.u_tol.
        gb = {k: v[b] for k, v in g.items()}
        e = {"phi": rel_err(g["phi"][b], mo["phi"], scale=1.0),
             "p": rel_err(g["p"][b], mo["p"], scale=scale_p)}
        du, res = u_abs_err(gb, mo), u_resolution(prm, mo["p"])
        print("replica", b, e, "|du| %.3e m/s = %.3f resolution units" % (du, du / res), flush=True)
        for k, v in e.items():
            assert v < FP32_TOL, (b, k, v)
        assert du < u_tol(prm, mo)


@pytest.mark.timeout(300)
def test_channel_leg_interior_against_periodic_oracle():
    from paper_2302_04120_amd import lbm
    nx, ny, steps = 16384, 2048, 20
    prm, ini = WL.channel(nx=nx, ny=ny)
    print_case(test="channel-leg", nx=nx, ny=ny, steps=steps)
    L = lbm.Lattice("channel", nx, ny, prec="fp32",
                    bc=(lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL),
                    flow=True, thermal=True)
    L.set_params(prm)
    L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    # the start state does not vary along x
    for k in ("rho", "ux", "uy", "T"):
        assert np.all(ini[k] == ini[k][:, :1])
    L.step(steps)
    assert L.reduce(("nonfinite",))["nonfinite"].sum() == 0
    g = {k: v[0] for k, v in L.macros().items()}
    lo, hi = steps + 2, nx - steps - 2
    inner = slice(lo, hi)
    for k, v in g.items():
        assert np.array_equal(v[:, inner], np.broadcast_to(v[:, lo:lo + 1], v[:, inner].shape)), k
    n8 = 8
    po = dict(prm, flux=np.full(n8, prm["q_s"]))
    o = O.Chan(n8, ny, po, bc_x="periodic", bc_y="walls", flow=True, thermal=True)
    o.init(ini["rho"][:, :n8], ini["ux"][:, :n8], ini["uy"][:, :n8], ini["T"][:, :n8])
    o.step(steps)
    mo = o.macros()
    c = prm["dx"] / prm["dt"]
    for x in (lo, 5000, 12345, hi - 1):
        gc = {k: v[:, x] for k, v in g.items()}
        oc = {k: v[:, 0] for k, v in mo.items()}
        rs = density_scale(oc["rho"], prm["rho_ref"], np.hypot(oc["ux"], oc["uy"]), c)
        umax = float(np.hypot(oc["ux"], oc["uy"]).max())
        e = {"rho": rel_err(gc["rho"], oc["rho"], prm["rho_ref"], scale=rs),
             "ux": rel_err(gc["ux"], oc["ux"], scale=umax),
             "uy": rel_err(gc["uy"], oc["uy"], scale=umax),
             "T": rel_err(gc["T"], oc["T"], prm["T_ref"])}
        print("column", x, e, flush=True)
        for k, v in e.items():
            assert v < FP32_TOL, (x, k, v)


@pytest.mark.timeout(300)
def test_fp64_bubble_leg_sampled():
    """The bench's FP64 leg: 256 replicas of the 256 x 256 bubble cell with
    the two-step kernel, 20 steps; sampled replicas against the oracle to
    FP64 rounding."""
    from paper_2302_04120_amd import lbm
    from gpu_cases import FP64_TOL
    batch, n, steps = 256, 256, 20
    prm, ini, _ = WL.bubble(n=n, batch=batch, seed=0)
    print_case(test="fp64-bubble-leg", batch=batch, steps=steps)
    L = lbm.Lattice("phase", n, n, batch=batch, prec="fp64")
    L.set_step_fusion(2)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    L.step(steps)
    assert L.reduce(("nonfinite",))["nonfinite"].sum() == 0
    g = L.macros(("phi", "p", "ux", "uy"))
    for b in (0, 129, 255):
        o = O.Phase(n, n, prm)
        o.init(ini["phi"][b], ini["p"][b], ini["ux"][b], ini["uy"][b])
        o.step(steps)
        mo = o.macros()
        umax = max(float(np.abs(mo["ux"]).max()), float(np.abs(mo["uy"]).max()))
        scale_p = max(float(np.abs(mo["p"]).max()), prm["sigma"] / prm["W"])
        e = {"phi": rel_err(g["phi"][b], mo["phi"], scale=1.0),
             "p": rel_err(g["p"][b], mo["p"], scale=scale_p),
             "ux": rel_err(g["ux"][b], mo["ux"], scale=umax),
             "uy": rel_err(g["uy"][b], mo["uy"], scale=umax)}
        print("replica", b, e, flush=True)
        for k, v in e.items():
            assert v < FP64_TOL, (b, k, v)

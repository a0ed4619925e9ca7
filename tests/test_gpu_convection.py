"""Natural convection in the App. D square cavity on the GPU: fixed-
temperature side walls, insulated top and bottom, Boussinesq force.  Parity
with the FP64 oracle over a transient, and the steady Ra = 1e4 state against
the oracle's stored run and the paper's Nusselt number."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

from cavity_ref import nusselt_hot_wall, nusselt_mean
from gpu_cases import print_case, rel_err

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _gpu_cavity(prm, ini, n, prec, batch=1):
    from paper_2302_04120_amd import lbm
    L = lbm.Lattice("channel", n, n, batch=batch, prec=prec,
                    bc=(lbm.BC_DIRICHLET, lbm.BC_DIRICHLET, lbm.BC_WALL, lbm.BC_WALL),
                    flow=True, thermal=True)
    L.set_params(prm)
    L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    return L


@pytest.mark.parametrize("prec,tol_T,tol_u", [("fp64", 1e-10, 1e-10), ("fp32", 1e-5, 1e-4)])
def test_cavity_parity_with_oracle(prec, tol_T, tol_u):
    """Ra = 1e4 cavity (65 x 65) from rest, 600 steps: GPU against the FP64
    oracle node by node (T relative to T_h - T_c, velocity to its maximum)."""
    prm, ini = WL.cavity(1e4)
    n = ini["rho"].shape[0]
    print_case(test="cavity-parity", prec=prec, n=n)
    L = _gpu_cavity(prm, ini, n, prec)
    L.step(600)
    g = {k: v[0] for k, v in L.macros().items()}
    o = O.Chan(n, n, prm, bc_x="walls_T", bc_y="walls", thermal=True)
    o.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    o.step(600)
    m = o.macros()
    dT = prm["Th"] - prm["Tc"]
    eT = rel_err(g["T"], m["T"], scale=dT)
    umax = max(np.abs(m["ux"]).max(), np.abs(m["uy"]).max())
    eu = max(rel_err(g["ux"], m["ux"], scale=umax), rel_err(g["uy"], m["uy"], scale=umax))
    print("cavity %s: T err %.2e (of dT), u err %.2e (of %.3e m/s)" % (prec, eT, eu, umax),
          flush=True)
    assert eT < tol_T
    assert eu < tol_u


def test_cavity_ra1e4_steady_nusselt():
    """The steady Ra = 1e4 cavity (40 000 steps, FP32 deviation storage):
    the mean and hot-wall Nusselt numbers equal the FP64 oracle's stored run
    (tests/golden/make_cavity.py) to 1e-4 and the paper's 2.242 (Table
    results_nat_conv; benchmark 2.243) to 0.1 %; mid-line profiles match the
    oracle's."""
    with open(os.path.join(HERE, "golden", "cavity_ra1e4_oracle.json")) as f:
        gold = json.load(f)
    prm, ini = WL.cavity(1e4)
    n = ini["rho"].shape[0]
    print_case(test="cavity-steady", steps=gold["steps"])
    L = _gpu_cavity(prm, ini, n, "fp32")
    L.step(gold["steps"])
    m = {k: v[0] for k, v in L.macros().items()}
    nu, nu0 = nusselt_mean(m["ux"], m["T"], prm), nusselt_hot_wall(m["T"], prm)
    print("Ra 1e4: Nu mean %.5f (oracle %.5f, paper 2.242), hot wall %.5f (oracle %.5f)" %
          (nu, gold["Nu_mean"], nu0, gold["Nu_hot_wall"]), flush=True)
    assert nu == pytest.approx(gold["Nu_mean"], rel=1e-4)
    assert nu0 == pytest.approx(gold["Nu_hot_wall"], rel=1e-4)
    assert nu == pytest.approx(2.242, rel=1e-3)
    mid = n // 2
    dT = prm["Th"] - prm["Tc"]
    uy_o = np.asarray(gold["row_mid_uy"])
    assert np.abs(m["uy"][mid] - uy_o).max() < 1e-3 * np.abs(uy_o).max()
    assert np.abs(m["T"][mid] - np.asarray(gold["row_mid_T"])).max() < 1e-4 * dT
    assert np.abs(m["ux"][:, mid] - np.asarray(gold["col_mid_ux"])).max() < \
        1e-3 * np.abs(gold["col_mid_ux"]).max()


@pytest.mark.timeout(300)
def test_cavity_ra1e6_steady_nusselt():
    """The steady Ra = 1e6 cavity (300 x 300, 260 000 steps, FP32 deviation
    storage): mean and hot-wall Nusselt numbers equal the FP64 oracle's stored
    run to 1e-4 and the paper's 8.805 (Table results_nat_conv, dimensional LBM;
    benchmark 8.800) to 0.3 %; mid-line profiles match the oracle's."""
    with open(os.path.join(HERE, "golden", "cavity_ra1e6_oracle.json")) as f:
        gold = json.load(f)
    prm, ini = WL.cavity(1e6)
    n = ini["rho"].shape[0]
    print_case(test="cavity-steady-1e6", n=n, steps=gold["steps"])
    L = _gpu_cavity(prm, ini, n, "fp32")
    L.step(gold["steps"])
    assert L.reduce(("nonfinite",))["nonfinite"].sum() == 0
    m = {k: v[0] for k, v in L.macros().items()}
    nu, nu0 = nusselt_mean(m["ux"], m["T"], prm), nusselt_hot_wall(m["T"], prm)
    print("Ra 1e6: Nu mean %.5f (oracle %.5f, paper 8.805), hot wall %.5f (oracle %.5f)" %
          (nu, gold["Nu_mean"], nu0, gold["Nu_hot_wall"]), flush=True)
    assert nu == pytest.approx(gold["Nu_mean"], rel=1e-4)
    assert nu0 == pytest.approx(gold["Nu_hot_wall"], rel=1e-4)
    assert nu == pytest.approx(8.805, rel=3e-3)
    mid = n // 2
    dT = prm["Th"] - prm["Tc"]
    uy_o = np.asarray(gold["row_mid_uy"])
    assert np.abs(m["uy"][mid] - uy_o).max() < 1e-3 * np.abs(uy_o).max()
    assert np.abs(m["T"][mid] - np.asarray(gold["row_mid_T"])).max() < 1e-4 * dT

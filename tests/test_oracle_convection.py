"""Pins of the oracle's natural-convection pieces (App. D): fixed-temperature
side walls (Eq. anti_BB_T on x), the Boussinesq force (Eq. buoyancy_force),
and the steady Ra = 1e4 cavity against the paper's printed Nusselt number."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL


HERE = os.path.dirname(os.path.abspath(__file__))


def _cavity(n, prm, T0):
    ch = O.Chan(n, n, prm, bc_x="walls_T", bc_y="walls", thermal=True)
    ch.init(np.full((n, n), prm["rho_ref"]), np.zeros((n, n)), np.zeros((n, n)),
            np.full((n, n), T0))
    return ch


def test_side_walls_pure_conduction_is_exactly_linear():
    """Without buoyancy the steady temperature between walls held at T_h and
    T_c (halfway walls, insulated top and bottom) is the linear conduction
    profile T = T_h + (T_c - T_h) x / L at the node centres x = (i + 1/2) dx;
    anti-bounce-back reproduces it exactly, and the fluid stays at rest."""
    prm, _ = WL.cavity(1e4, n=12)
    prm = dict(prm, beta_T=0.0)
    n = 12
    ch = _cavity(n, prm, prm["Tc"])
    ch.step(6000)
    m = ch.macros()
    x = (np.arange(n) + 0.5) * prm["dx"]
    T_lin = prm["Th"] + (prm["Tc"] - prm["Th"]) * x / prm["L"]
    assert np.abs(m["T"] - T_lin[None, :]).max() < 1e-9 * (prm["Th"] - prm["Tc"])
    assert np.abs(m["ux"]).max() < 1e-14 and np.abs(m["uy"]).max() < 1e-14


def test_boussinesq_force_at_uniform_temperature_is_a_body_force():
    """At a uniform temperature T_ref + dT the Boussinesq force is the constant
    body force -rho_ref beta dT g: a periodic channel driven that way evolves
    exactly like one driven by that body force."""
    nx, ny, dT = 8, 12, 5.0
    base, _ = WL.cavity(1e4, n=ny)
    beta, g = base["beta_T"], (-9.81, 0.0)
    prm = dict(base, flux=np.zeros(nx), inlet_u=np.zeros(ny), inlet_T=np.full(ny, base["T_ref"]))
    runs = []
    for mode in ("buoyancy", "body"):
        p = dict(prm, beta_T=beta if mode == "buoyancy" else 0.0, gravity=g,
                 Fx=0.0 if mode == "buoyancy" else -prm["rho_ref"] * beta * dT * g[0])
        ch = O.Chan(nx, ny, p, bc_x="periodic", bc_y="walls", thermal=True)
        ch.init(np.full((ny, nx), prm["rho_ref"]), np.zeros((ny, nx)), np.zeros((ny, nx)),
                np.full((ny, nx), prm["T_ref"] + dT))
        ch.step(400)
        runs.append(ch.macros())
    a, b = runs
    assert np.abs(a["ux"]).max() > 1e-6  # the force drives a flow
    np.testing.assert_allclose(a["ux"], b["ux"], rtol=1e-11, atol=1e-18)
    np.testing.assert_allclose(a["T"], b["T"], rtol=1e-14)


def test_cavity_centro_symmetry():
    """With T_ref midway between the wall temperatures, the cavity problem is
    invariant under a half-turn combined with T -> T_h + T_c - T (the force
    changes sign with T - T_ref).  From a symmetric start (rest, T = T_ref)
    every field keeps that symmetry; the hot side rises."""
    prm, _ = WL.cavity(1e4, n=16)
    prm = dict(prm, T_ref=0.5 * (prm["Th"] + prm["Tc"]))
    ch = _cavity(16, prm, prm["T_ref"])
    ch.step(1500)
    m = ch.macros()
    rot = lambda a: a[::-1, ::-1]
    dT = prm["Th"] - prm["Tc"]
    assert np.abs(m["T"] + rot(m["T"]) - (prm["Th"] + prm["Tc"])).max() < 1e-11 * dT
    umax = np.abs(m["ux"]).max()
    assert umax > 1e-5
    assert np.abs(m["ux"] + rot(m["ux"])).max() < 1e-9 * umax
    assert np.abs(m["uy"] + rot(m["uy"])).max() < 1e-9 * umax
    assert m["uy"][8, 0] > 0 > m["uy"][8, -1]


def test_cavity_ra1e4_nusselt_against_paper():
    """The stored FP64 oracle run of the App. D cavity at Ra = 1e4 (written by
    tests/golden/make_cavity.py) is steady and its mean Nusselt number is the
    paper's 2.242 (Table results_nat_conv, dimensional LBM; benchmark 2.243)
    to within 0.1 %; the hot-wall value agrees with it to 0.1 %."""
    with open(os.path.join(HERE, "golden", "cavity_ra1e4_oracle.json")) as f:
        g = json.load(f)
    assert g["Nu_change_last_interval"] < 1e-5
    assert g["Nu_mean"] == pytest.approx(2.242, rel=1e-3)
    assert g["Nu_mean"] == pytest.approx(2.243, rel=2e-3)
    assert g["Nu_hot_wall"] == pytest.approx(g["Nu_mean"], rel=1e-3)
    # the flow turns clockwise with the hot wall on the left: up near it, down at the cold one
    uy = np.asarray(g["row_mid_uy"])
    assert uy[2] > 0 > uy[-3]


def test_cavity_ra1e6_nusselt_against_paper():
    """The stored FP64 oracle run at Ra = 1e6 (300 x 300, 260 000 steps,
    tests/golden/make_cavity.py 1e6) is steady and its mean Nusselt number is
    the paper's 8.805 (Table results_nat_conv, dimensional LBM) and the
    benchmark's 8.800 to within 0.3 %; hot-wall and mean values agree to
    0.5 %; the boundary layers make the mid-height vertical velocity peak
    near the walls."""
    with open(os.path.join(HERE, "golden", "cavity_ra1e6_oracle.json")) as f:
        g = json.load(f)
    assert g["Nu_change_last_interval"] < 5e-4 * g["Nu_mean"]
    assert g["Nu_mean"] == pytest.approx(8.805, rel=3e-3)
    assert g["Nu_mean"] == pytest.approx(8.800, rel=3e-3)
    assert g["Nu_hot_wall"] == pytest.approx(g["Nu_mean"], rel=5e-3)
    uy = np.asarray(g["row_mid_uy"])
    n = uy.size
    assert uy[: n // 10].max() == pytest.approx(uy.max())  # peak within a tenth of the hot wall
    assert uy[-(n // 10):].min() == pytest.approx(uy.min())

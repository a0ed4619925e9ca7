"""GPU (HIP, through the C ABI) versus FP64 oracle, element by element.

Sizes: small grids that span several 64 x 4 tiles with ragged edges in both
directions, a few hundred steps; plus the paper-shaped configurations at
their full size for a bounded number of steps.
"""
import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

from gpu_cases import FP32_TOL, FP64_TOL, channel_pair, phase_pair, print_case, rel_err

pytestmark = pytest.mark.gpu


def _chan_fields_check(g, o, prm, tol, thermal=True):
    errs = {"rho": rel_err(g["rho"], o["rho"], prm["rho_ref"]),
            "ux": rel_err(g["ux"], o["ux"]),
            "uy": rel_err(g["uy"], o["uy"])}
    if thermal:
        errs["T"] = rel_err(g["T"], o["T"], prm["T_ref"])
    print("errors", errs, flush=True)
    for k, v in errs.items():
        assert v < tol, (k, v)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_channel_inlet_outlet_flux_walls(prec, tol):
    """D2Q9 MRT + D2Q5 two-rate, velocity inlet, pressure outlet, flux walls with
    a spatial square-wave flux and temporal oscillation; ragged 150 x 22 grid."""
    nx, ny = 150, 22
    print_case(test="channel_io", prec=prec, nx=nx, ny=ny)
    prm, ini = WL.channel(nx=nx, ny=ny, dx=5e-5, tau_ratio=0.6, oscillating=True)
    prm["flux"] = 1e4 * (1 + np.sign(np.sin(2 * np.pi * np.arange(nx) / 40.0)))
    prm["flux_omega"] = 2 * np.pi / (150 * prm["dt"])
    g, o, _, _ = channel_pair(prm, ini, nx, ny, 300, prec)
    _chan_fields_check(g, o, prm, tol)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
@pytest.mark.parametrize("mrt", [0, 1])
def test_channel_periodic_forced(prec, tol, mrt):
    """Force-driven flow between halfway walls, periodic in x (App. C shape),
    BGK and MRT, from a seeded random initial velocity."""
    nx, ny = 70, 30
    print_case(test="channel_periodic", prec=prec, mrt=mrt)
    nu, rho = 8.382e-7, 996.279
    dx = 1e-5
    dt = 0.3 * dx * dx / (3 * nu)
    prm = dict(dx=dx, dt=dt, rho_ref=rho, nu=nu, Fx=2e2, Fy=-50.0, flow_mrt=mrt)
    g0 = WL.rng(21)
    ini = dict(rho=rho + g0.uniform(-0.5, 0.5, (ny, nx)), ux=g0.uniform(-1e-3, 1e-3, (ny, nx)),
               uy=g0.uniform(-1e-3, 1e-3, (ny, nx)))
    g, o, _, _ = channel_pair(prm, ini, nx, ny, 400, prec, bc_x="periodic", bc_y="walls",
                              thermal=False)
    _chan_fields_check(g, o, prm, tol, thermal=False)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_channel_thermal_only_bgk_source(prec, tol):
    """Frozen flow, D2Q5 BGK with volumetric source and flux walls, periodic x."""
    nx, ny = 66, 9
    print_case(test="thermal_only", prec=prec)
    dx, alpha = 1e-5, 1e-7
    dt = 0.2 * dx * dx / (3 * alpha)
    g0 = WL.rng(5)
    prm = dict(dx=dx, dt=dt, rho_ref=1000.0, alpha=alpha, rho_cp=4e6, T_ref=300.0,
               qdot=0.5, thermal_mrt=0, flux=g0.uniform(0, 2e4, nx))
    ini = dict(rho=np.full((ny, nx), 1000.0), ux=np.full((ny, nx), 2e-3),
               uy=np.zeros((ny, nx)), T=300 + g0.uniform(-1, 1, (ny, nx)))
    g, o, _, _ = channel_pair(prm, ini, nx, ny, 250, prec, bc_x="periodic", bc_y="walls",
                              flow=False)
    assert rel_err(g["T"], o["T"], 300.0) < tol


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_channel_nusselt_diagnostics(prec, tol):
    nx, ny = 100, 20
    print_case(test="nusselt", prec=prec)
    prm, ini = WL.channel(nx=nx, ny=ny, dx=5e-5, tau_ratio=0.6)
    g, o, L, oc = channel_pair(prm, ini, nx, ny, 500, prec)
    Tb, Tw, Nu, nm, tout = L.nusselt(nx // 2)
    oTb, oTw, oNu = oc.nusselt()
    assert rel_err(Tb, oTb, 300.0) < tol
    assert rel_err(Nu, oNu) < 100 * tol
    assert nm == pytest.approx(oNu[nx // 2:].mean(), rel=100 * tol)
    assert tout == pytest.approx(oTb[-1], rel=tol)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_phase_bubble_ragged(prec, tol):
    """Two-phase bubble (C3 properties, 43 000 density ratio) on a ragged
    80 x 38 periodic grid: phi, pressure and velocity against the oracle."""
    nx, ny = 80, 38
    print_case(test="phase_bubble", prec=prec)
    prm, ini, _ = WL.bubble(n=80, radii=(12,), batch=1, seed=3)
    ini = {k: v[:, :ny, :].copy() for k, v in ini.items()}
    prm["normal_eps"] = 1e-6 / prm["dx"]
    g, o, _, _ = phase_pair(prm, ini, nx, ny, 200, prec)
    errs = {k: rel_err(g[k], o[k]) for k in ("phi", "p", "ux", "uy")}
    errs["rho"] = rel_err(g["rho"], o["rho"], prm["rho_g"])
    print("errors", errs, flush=True)
    for k, v in errs.items():
        assert v < (tol if k != "uy" and k != "ux" else 10 * tol), (k, v)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_phase_layered_walls(prec, tol):
    """Layered two-phase channel with halfway walls and zeta-linear viscosity
    (C4 shape, narrow periodic x)."""
    print_case(test="phase_layered", prec=prec)
    prm, ini, _ = WL.layered(nx=4, ny=96, dx=5e-6, dt=2.5e-7, W_nodes=6, seed=2)
    prm["normal_eps"] = 1e-6 / prm["dx"]
    g, o, _, _ = phase_pair(prm, ini, 4, 96, 400, prec, bc_y="walls")
    errs = {k: rel_err(g[k], o[k]) for k in ("phi", "p", "ux")}
    print("errors", errs, flush=True)
    for k, v in errs.items():
        assert v < tol, (k, v)


def test_phase_bgk_and_printed_qy():
    """Alternative collision choices: BGK for z, and the printed anisotropic
    q_y rate (FP64)."""
    for variant in ({"z_mrt": 0}, {"qy_printed": 1}):
        print_case(test="phase_variant", **variant)
        prm, ini, _ = WL.bubble(n=40, radii=(8,), batch=1, seed=7, nu_g=1e-5)
        prm.update(variant)
        prm["normal_eps"] = 1e-6 / prm["dx"]
        g, o, _, _ = phase_pair(prm, ini, 40, 40, 150, "fp64")
        for k in ("phi", "p", "ux"):
            assert rel_err(g[k], o[k]) < FP64_TOL, (variant, k)


def test_d1_slab_matches_oracle_and_analytic():
    """C1: D1Q2 and D1Q3 with source, wet Dirichlet ends, 2e5 steps, FP64."""
    from paper_2302_04120_amd import lbm
    prm, T0 = WL.slab_1d(seed=0)
    x = np.arange(101) * prm["dx"]
    Ta = 300 + prm["qvol"] * x * (prm["L"] - x) / (2 * prm["k"])
    for lat, q in (("d1q2", 2), ("d1q3", 3)):
        print_case(test="d1", lattice=lat)
        L = lbm.Lattice(lat, 101, prec="fp64")
        L.set_params(prm)
        L.init(T=T0)
        L.step(200000)
        T = L.macros(("T",))["T"][0, 0]
        To = O.d1_run(q, 101, prm["dx"], prm["dt"], prm["alpha"], prm["qdot"], 300, 300, T0, 200000)
        assert np.abs(T - To).max() < 1e-9
        assert np.abs(T - Ta).max() < 1e-6


def test_phase_mass_conserved_fp32_exactly():
    """R-MASS: with FP32 storage the global order parameter is conserved to
    FP64 reduction rounding over 2000 steps (bubble, periodic)."""
    from paper_2302_04120_amd import lbm
    print_case(test="rmass")
    prm, ini, _ = WL.bubble(n=64, radii=(16, 20), batch=2, seed=1)
    L = lbm.Lattice("phase", 64, 64, batch=2, prec="fp32")
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    m0 = L.reduce(("phase",))["phase"]
    L.step(2000)
    m1 = L.reduce(("phase",))["phase"]
    rel = np.abs(m1 - m0) / m0
    print("mass drift", rel, flush=True)
    assert rel.max() < 1e-12


def test_batched_replicas_independent():
    """Replicas of a batch evolve independently: replica 1 of a batch equals a
    single-replica oracle run of its own inputs."""
    print_case(test="batch")
    prm, ini, _ = WL.bubble(n=48, radii=(10, 14, 9), batch=3, seed=11)
    prm["normal_eps"] = 1e-6 / prm["dx"]
    g, o, _, _ = phase_pair(prm, ini, 48, 48, 100, "fp64", replica=1)
    for k in ("phi", "p", "ux"):
        assert rel_err(g[k], o[k]) < FP64_TOL, k


def test_save_load_resume_bit_identical():
    from paper_2302_04120_amd import lbm
    print_case(test="resume")
    prm, ini, _ = WL.bubble(n=64, radii=(12,), batch=1, seed=2)
    a = lbm.Lattice("phase", 64, 64, prec="fp32")
    a.set_params(prm)
    a.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    a.step(50)
    blob = a.save_state()
    a.step(70)
    ra = a.macros()
    b = lbm.Lattice("phase", 64, 64, prec="fp32")
    b.set_params(prm)
    b.load_state(blob)
    assert b.t == 50
    b.step(70)
    rb = b.macros()
    for k in ra:
        assert np.array_equal(ra[k], rb[k]), k
    with pytest.raises(lbm.LbmError):
        b.load_state(blob[:100])


def test_error_paths_on_device():
    from paper_2302_04120_amd import lbm
    L = lbm.Lattice("channel", 16, 8, prec="fp32", bc=(0, 0, 1, 1))
    with pytest.raises(lbm.LbmError) as e:
        L.set_params(dict(dx=1e-5, dt=1e-4, rho_ref=1000.0, nu=0.0))
    assert e.value.status == lbm.LBM_E_TAU
    with pytest.raises(lbm.LbmError) as e:
        L.step(1)
    assert e.value.status == lbm.LBM_E_STATE
    L.set_params(dict(dx=1e-5, dt=1e-4, rho_ref=1000.0, nu=1e-6))
    L.init(np.full((8, 16), 1000.0))
    # a non-finite value planted through the state blob is reported
    blob = bytearray(L.save_state())
    import struct
    hdr = 4 + 4 + 6 * 4 + 8 + 8 + 8 + 8
    blob[hdr:hdr + 4] = struct.pack("<f", float("nan"))
    L.load_state(bytes(blob))
    with pytest.raises(lbm.LbmError) as e:
        L.reduce()
    assert e.value.status == lbm.LBM_E_NONFINITE


# ---------------------------------------------------------------- full sizes
def test_full_size_channel_c2_sampled():
    """C2 at its full 800 x 40 size, FP32-dev, 200 steps, all nodes compared."""
    print_case(test="c2_full")
    prm, ini = WL.channel(nx=800, ny=40, tau_ratio=0.64, oscillating=True)
    g, o, _, _ = channel_pair(prm, ini, 800, 40, 200, "fp32")
    _chan_fields_check(g, o, prm, FP32_TOL)


def test_full_size_bubble_replica_sampled():
    """C3 cell at its full 256 x 256 size inside a batch of 8 replicas (the
    bench's launch shape), FP32-dev, 60 steps; replica 5 against the oracle."""
    print_case(test="c3_full")
    prm, ini, _ = WL.bubble(n=256, batch=8, seed=0)
    prm["normal_eps"] = 1e-6 / prm["dx"]
    g, o, _, _ = phase_pair(prm, ini, 256, 256, 60, "fp32", replica=5)
    for k in ("phi", "p"):
        assert rel_err(g[k], o[k]) < FP32_TOL, k
    assert rel_err(g["ux"], o["ux"]) < 10 * FP32_TOL

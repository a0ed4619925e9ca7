"""Degenerate grid sizes of the two-phase lattice against the FP64 oracle:
replicas of one node, one row or one column, where the periodic neighbours
of a node are the node itself or its only neighbour, and single rows between
walls, where both walls reflect into the same row.  A tile of the kernel then
holds a few valid nodes and its ring wraps onto them.  Both the single-step
kernel and the many-steps kernel (one tile) run every case; FP64 to
rounding, and the phi sum to 1e-13."""
import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

from gpu_cases import FP64_TOL, print_case, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fusion", [1, 3])
@pytest.mark.parametrize("nx,ny,walls", [(1, 1, False), (1, 5, False), (3, 2, False),
                                         (2, 1, True), (5, 2, True), (7, 3, True)])
def test_tiny_phase_grids(nx, ny, walls, fusion):
    from paper_2302_04120_amd import lbm
    steps, batch = 10, 2
    prm, _, _ = WL.bubble(n=nx, ny=ny, radii=(1,), batch=1, seed=1)
    g = WL.rng(nx * 10 + ny)
    ini = {"phi": g.uniform(0.2, 0.8, (batch, ny, nx)),
           "p": 10 * g.uniform(-1, 1, (batch, ny, nx)),
           "ux": 1e-3 * g.uniform(-1, 1, (batch, ny, nx)),
           "uy": 1e-3 * g.uniform(-1, 1, (batch, ny, nx))}
    print_case(test="tiny-phase", nx=nx, ny=ny, walls=walls, fusion=fusion)
    bc = (0, 0, lbm.BC_WALL, lbm.BC_WALL) if walls else (0, 0, 0, 0)
    L = lbm.Lattice("phase", nx, ny, batch=batch, prec="fp64", bc=bc)
    L.set_step_fusion(fusion)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    L.step(steps)
    m = L.macros(("phi", "p", "ux", "uy"))
    for b in range(batch):
        o = O.Phase(nx, ny, prm, bc_y="walls" if walls else "periodic")
        o.init(ini["phi"][b], ini["p"][b], ini["ux"][b], ini["uy"][b])
        s0 = o.macros()["phi"].sum()
        o.step(steps)
        mo = o.macros()
        umax = max(float(np.abs(mo["ux"]).max()), float(np.abs(mo["uy"]).max()))
        scale_p = max(float(np.abs(mo["p"]).max()), prm["sigma"] / prm["W"])
        errs = {"phi": rel_err(m["phi"][b], mo["phi"], scale=1.0),
                "p": rel_err(m["p"][b], mo["p"], scale=scale_p),
                "ux": rel_err(m["ux"][b], mo["ux"], scale=umax),
                "uy": rel_err(m["uy"][b], mo["uy"], scale=umax)}
        print("replica", b, errs, flush=True)
        for k, v in errs.items():
            assert v < FP64_TOL, (b, k, v)
        assert abs(m["phi"][b].sum() - s0) < 1e-13 * max(abs(s0), 1.0)


KINDS = {"periodic": 0, "walls": 1}


@pytest.mark.parametrize("nx,ny,nz,bcs", [(1, 1, 1, ("periodic",) * 3),
                                          (2, 3, 1, ("walls", "walls", "periodic")),
                                          (1, 2, 3, ("periodic", "periodic", "walls"))])
def test_tiny_d3q19_grids(nx, ny, nz, bcs):
    """D3Q19 MRT with body force on boxes of one to six nodes, FP64, 20 steps."""
    from paper_2302_04120_amd import lbm
    steps, batch = 20, 2
    prm, ini = WL.box3d(nx, ny, nz, batch=batch, seed=5, F=(40.0, -25.0, 15.0), mrt=True)
    print_case(test="tiny-d3q19", nx=nx, ny=ny, nz=nz, bcs=bcs)
    bx, by, bz = (KINDS[b] for b in bcs)
    L = lbm.Lattice("d3q19", nx, ny, batch=batch, prec="fp64", bc=(bx, bx, by, by), nz=nz,
                    bc_z=(bz, bz))
    L.set_params(prm)
    L.init3d(ini["rho"], ini["ux"], ini["uy"], ini["uz"])
    L.step(steps)
    g = L.macros()
    c = prm["dx"] / prm["dt"]
    for b in range(batch):
        o = O.D3(nx, ny, nz, prm, bc_x=bcs[0], bc_y=bcs[1], bc_z=bcs[2], mrt=True)
        o.init(ini["rho"][b], ini["ux"][b], ini["uy"][b], ini["uz"][b])
        o.step(steps)
        m = o.macros()
        umax = max(float(np.abs(m[k]).max()) for k in ("ux", "uy", "uz"))
        rs = max(float(np.abs(m["rho"] - prm["rho_ref"]).max()), 3 * prm["rho_ref"] * umax / c)
        errs = {"rho": rel_err(g["rho"][b], m["rho"], scale=rs)}
        for k in ("ux", "uy", "uz"):
            errs[k] = rel_err(g[k][b], m[k], scale=umax)
        print("replica", b, errs, flush=True)
        for k, v in errs.items():
            assert v < FP64_TOL, (b, k, v)


@pytest.mark.parametrize("nx,ny,nz,bcs", [(1, 1, 1, ("periodic",) * 3),
                                          (3, 2, 2, ("walls", "periodic", "walls"))])
def test_tiny_phase3d_grids(nx, ny, nz, bcs):
    """The 3D two-phase step on boxes of one and twelve nodes, FP64, 10 steps:
    the LDS halo of phi wraps onto the node itself or mirrors at the walls."""
    from paper_2302_04120_amd import lbm
    steps = 10
    prm, ini = WL.bubble3d(n=nx, ny=ny, nz=nz, R_nodes=1.0, seed=2, u_noise=0.02)
    print_case(test="tiny-phase3d", nx=nx, ny=ny, nz=nz, bcs=bcs)
    bx, by, bz = (KINDS[b] for b in bcs)
    L = lbm.Lattice("phase3d", nx, ny, batch=1, prec="fp64", bc=(bx, bx, by, by), nz=nz,
                    bc_z=(bz, bz))
    L.set_params(prm)
    L.init3d(ini["p"], ini["ux"], ini["uy"], ini["uz"], ini["phi"])
    L.step(steps)
    g = {k: v[0] for k, v in L.macros().items()}
    o = O.Phase3(nx, ny, nz, prm, bc_x=bcs[0], bc_y=bcs[1], bc_z=bcs[2])
    o.init(ini["phi"][0], ini["p"][0], ini["ux"][0], ini["uy"][0], ini["uz"][0])
    o.step(steps)
    m = o.macros()
    umax = max(float(np.abs(m[k]).max()) for k in ("ux", "uy", "uz"))
    scale_p = max(float(np.abs(m["p"]).max()), prm["sigma"] / prm["W"])
    errs = {"phi": rel_err(g["phi"], m["phi"], scale=1.0), "p": rel_err(g["p"], m["p"], scale=scale_p)}
    for k in ("ux", "uy", "uz"):
        errs[k] = rel_err(g[k], m[k], scale=umax)
    print(errs, flush=True)
    for k, v in errs.items():
        assert v < FP64_TOL, (k, v)


@pytest.mark.parametrize("nx,ny", [(2, 1), (3, 2), (5, 1)])
def test_tiny_heated_channel_grids(nx, ny):
    """The heated channel (D2Q9 MRT flow, D2Q5 thermal, velocity inlet next
    to the pressure outlet, flux walls that reflect into the same row when ny
    = 1, oscillating flux), FP64, 30 steps.  Velocity errors are taken on the
    scale of |u| (u_y is zero to rounding in one-row channels)."""
    from gpu_cases import channel_pair, density_scale
    print_case(test="tiny-channel", nx=nx, ny=ny)
    prm, ini = WL.channel(nx=nx, ny=ny, dx=5e-5, tau_ratio=0.6, oscillating=True)
    g, o, _, _ = channel_pair(prm, ini, nx, ny, 30, "fp64")
    c = prm["dx"] / prm["dt"]
    umax = float(np.hypot(o["ux"], o["uy"]).max())
    rs = density_scale(o["rho"], prm["rho_ref"], np.hypot(o["ux"], o["uy"]), c)
    errs = {"rho": rel_err(g["rho"], o["rho"], prm["rho_ref"], scale=rs),
            "ux": rel_err(g["ux"], o["ux"], scale=umax),
            "uy": rel_err(g["uy"], o["uy"], scale=umax),
            "T": rel_err(g["T"], o["T"], prm["T_ref"])}
    print(errs, flush=True)
    for k, v in errs.items():
        assert v < FP64_TOL, (k, v)

"""The D3Q19 kernel (3D dimensional MRT / BGK with Guo forcing and halfway
walls) against the FP64 oracle, node by node, through the C ABI.

Grids span several 64 x 4 tiles with ragged x and y tails, several z planes
and replicas; every boundary combination the library accepts appears.  At the
benchmark's size (256^3, FP32) the whole field is checked against the oracle
by building an input that repeats an 8 x 8 cell in x and y: the exact
solution then repeats too, and the oracle runs the 8 x 8 x 256 cell."""
import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

from gpu_cases import FP32_TOL, FP64_TOL, print_case, rel_err

pytestmark = pytest.mark.gpu

KINDS = {"periodic": 0, "walls": 1}


def _gpu(prm, ini, nx, ny, nz, batch, prec, bcs, steps, graph_steps=64):
    from paper_2302_04120_amd import lbm
    bx, by, bz = (KINDS[b] for b in bcs)
    L = lbm.Lattice("d3q19", nx, ny, batch=batch, prec=prec, bc=(bx, bx, by, by), nz=nz,
                    bc_z=(bz, bz))
    L.set_graph_steps(graph_steps)
    L.set_params(prm)
    L.init3d(ini["rho"], ini["ux"], ini["uy"], ini["uz"])
    L.step(steps)
    return L


def _oracle(prm, ini, b, nx, ny, nz, bcs, steps, mrt):
    o = O.D3(nx, ny, nz, prm, bc_x=bcs[0], bc_y=bcs[1], bc_z=bcs[2], mrt=mrt)
    o.init(ini["rho"][b], ini["ux"][b], ini["uy"][b], ini["uz"][b])
    o.step(steps)
    return o.macros()


def _errors(g, m, prm):
    c = prm["dx"] / prm["dt"]
    umax = max(np.abs(m[k]).max() for k in ("ux", "uy", "uz"))
    # density travels in FP32 deviations of size ~ rho 3 |u| / c (see gpu_cases)
    rs = max(np.abs(m["rho"] - prm["rho_ref"]).max(), 3 * prm["rho_ref"] * umax / c)
    e = {"rho": rel_err(g["rho"], m["rho"], scale=rs)}
    for k in ("ux", "uy", "uz"):
        e[k] = rel_err(g[k], m[k], scale=umax)
    return e


CASES = [
    # nx, ny, nz, batch, (bc x, y, z), mrt
    (70, 9, 5, 2, ("periodic", "periodic", "periodic"), True),
    (70, 9, 5, 1, ("periodic", "walls", "walls"), True),
    (33, 14, 6, 1, ("walls", "walls", "walls"), True),
    (70, 9, 5, 1, ("walls", "periodic", "walls"), False),
    (64, 4, 3, 2, ("periodic", "walls", "periodic"), False),
]


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
@pytest.mark.parametrize("nx,ny,nz,batch,bcs,mrt", CASES)
def test_d3q19_parity(nx, ny, nz, batch, bcs, mrt, prec, tol):
    steps = 60
    prm, ini = WL.box3d(nx, ny, nz, batch=batch, seed=nx + ny + nz, F=(40.0, -25.0, 15.0),
                        mrt=mrt)
    prm["omega_e"] = 1.2 / prm["dt"]
    prm["omega_eps"] = 0.8 / prm["dt"]
    print_case(test="d3q19-parity", nx=nx, ny=ny, nz=nz, batch=batch, bcs=bcs, mrt=mrt, prec=prec)
    L = _gpu(prm, ini, nx, ny, nz, batch, prec, bcs, steps)
    g = L.macros()
    for b in range(batch):
        m = _oracle(prm, ini, b, nx, ny, nz, bcs, steps, mrt)
        e = _errors({k: v[b] for k, v in g.items()}, m, prm)
        print("replica", b, e, flush=True)
        for k, v in e.items():
            assert v < tol, (b, k, v)
    red = L.reduce(("mass", "nonfinite"))
    assert red["nonfinite"].sum() == 0


def test_d3q19_mass_conservation_and_graph_replay():
    """FP64, walls on all sides: the total mass stays at its initial value to
    rounding over 500 steps, and graph replay reproduces step-by-step launches
    to the bit."""
    nx, ny, nz = 40, 12, 10
    prm, ini = WL.box3d(nx, ny, nz, seed=3, F=(10.0, 0.0, 0.0))
    bcs = ("walls", "walls", "walls")
    print_case(test="d3q19-mass-graph")
    a = _gpu(prm, ini, nx, ny, nz, 1, "fp64", bcs, 0, graph_steps=0)
    m0 = a.reduce(("mass",))["mass"][0]
    a.step(500)
    assert a.reduce(("mass",))["mass"][0] == pytest.approx(m0, rel=1e-13)
    b = _gpu(prm, ini, nx, ny, nz, 1, "fp64", bcs, 0, graph_steps=16)
    b.step(500)
    assert a.save_state() == b.save_state()
    for prec in ("fp32",):
        a = _gpu(prm, ini, nx, ny, nz, 1, prec, bcs, 77, graph_steps=0)
        b = _gpu(prm, ini, nx, ny, nz, 1, prec, bcs, 77, graph_steps=8)
        assert a.save_state() == b.save_state()


def test_d3q19_save_load_round_trip():
    nx, ny, nz = 24, 8, 6
    prm, ini = WL.box3d(nx, ny, nz, seed=4)
    bcs = ("periodic", "walls", "periodic")
    print_case(test="d3q19-save-load")
    a = _gpu(prm, ini, nx, ny, nz, 1, "fp32", bcs, 10)
    blob = a.save_state()
    a.step(15)
    b = _gpu(prm, ini, nx, ny, nz, 1, "fp32", bcs, 0)
    b.load_state(blob)
    assert b.t == 10
    b.step(15)
    assert a.save_state() == b.save_state()


def test_d3q19_poiseuille_between_walls():
    """FP32 storage reaches the oracle-pinned steady profile: the parabola
    plus the slip F dx^2 (16 Lambda - 3)/(24 rho nu), Lambda = 1/12 for the
    MRT rates of Sec. 3 (walls normal to z, force along x)."""
    from paper_2302_04120_amd import lbm
    n, rho, nu, dx = 16, 1000.0, 1e-6, 1e-4
    dt = 0.3 * dx * dx / (3 * nu)
    F = 0.05
    prm = dict(dx=dx, dt=dt, rho_ref=rho, nu=nu, F=(F, 0.0, 0.0), flow_mrt=1)
    print_case(test="d3q19-poiseuille")
    L = lbm.Lattice("d3q19", 64, 4, prec="fp32", bc=(0, 0, 0, 0), nz=n, bc_z=(1, 1))
    L.set_params(prm)
    sh = (1, n, 4, 64)
    L.init3d(np.full(sh, rho))
    H = n * dx
    L.step(int(7 * H * H / nu / dt))
    ux = L.macros(("ux",))["ux"][0]
    s = (np.arange(n) + 0.5) * dx
    exact = F / (2 * rho * nu) * s * (H - s) + F * dx * dx * (16 / 12 - 3) / (24 * rho * nu)
    err = np.abs(ux - exact[:, None, None]).max() / exact.max()
    print("Poiseuille max rel error %.2e" % err, flush=True)
    assert err < 1e-4


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("fp64", FP64_TOL)])
def test_d3q19_bench_size_whole_field(prec, tol):
    """The benchmark's box, 256^3 periodic, MRT with forcing, 20 steps: an
    input that repeats an 8 x 8 cell in x and y has an exact solution that
    repeats too, so every node of the GPU field is compared with the FP64
    oracle run on the 8 x 8 x 256 cell."""
    n, cell, steps = 256, 8, 20
    prm, ini = WL.box3d(n, n, n, seed=12, period=(cell, cell), F=(30.0, 20.0, -10.0))
    prm["omega_e"] = 1.1 / prm["dt"]
    print_case(test="d3q19-bench-size", n=n, prec=prec)
    L = _gpu(prm, ini, n, n, n, 1, prec, ("periodic",) * 3, steps)
    assert L.reduce(("nonfinite",))["nonfinite"].sum() == 0
    g = {k: v[0] for k, v in L.macros().items()}
    cini = {k: v[:, :, :cell, :cell] for k, v in ini.items()}
    m = _oracle(prm, cini, 0, cell, cell, n, ("periodic",) * 3, steps, True)
    reps = (1, n // cell, n // cell)
    e = _errors(g, {k: np.tile(v, reps) for k, v in m.items()}, prm)
    print("errors", e, flush=True)
    for k, v in e.items():
        assert v < tol, (k, v)

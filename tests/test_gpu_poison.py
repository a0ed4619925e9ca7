"""Every output slot of a step is written: the buffer a step writes into is
filled with NaN bytes (0xFF, a NaN in FP32 and FP64) before the step, and the
state after the step must hold no non-finite value and equal, bit for bit,
the state of a twin run whose buffers were never poisoned.  A population, a
(phi u) plane or a boundary rule that left a slot unwritten would carry the
NaN into the state.  Covered: the heated channel (inlet, outlet, flux walls),
the two-phase single-step, two-step and many-steps kernels (periodic and
walls), D3Q19 and the 3D two-phase step (whose phi plane is poisoned too)."""
import numpy as np
import pytest

from paper_2302_04120_amd import workloads as WL

from gpu_cases import print_case

pytestmark = pytest.mark.gpu

PAD = 16448  # extra elements per plane of the library's layout


def _pop_bytes(L, nplanes):
    N = L.batch * L.nz * L.ny * L.nx
    P = (N + 63) // 64 * 64 + PAD
    es = 4 if L.prec == "fp32" else 8
    return (nplanes * P * es + 255) // 256 * 256, P * es


def _poison_next(L, nplanes, extra=()):
    """Fill the buffer the next step writes (B while the state is in A, right
    after initialisation) and any extra (offset, length) ranges."""
    import torch
    torch.cuda.synchronize()
    pb, _ = _pop_bytes(L, nplanes)
    L.buf[pb:2 * pb].fill_(255)
    for off, n in extra:
        L.buf[off:off + n].fill_(255)
    torch.cuda.synchronize()


def _check(L, twin, steps):
    L.step(steps)
    twin.step(steps)
    assert L.reduce(("nonfinite",))["nonfinite"].sum() == 0
    assert L.save_state() == twin.save_state()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_channel_writes_every_slot(prec):
    from paper_2302_04120_amd import lbm
    print_case(test="poison-channel", prec=prec)
    prm, ini = WL.channel(nx=150, ny=22, dx=5e-5, tau_ratio=0.6, oscillating=True)

    def make():
        L = lbm.Lattice("channel", 150, 22, prec=prec,
                        bc=(lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL),
                        flow=True, thermal=True)
        L.set_graph_steps(0)
        L.set_params(prm)
        L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
        return L

    L, twin = make(), make()
    _poison_next(L, 9 + 5)
    _check(L, twin, 1)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("fusion,nx,ny,walls,steps", [(1, 70, 37, False, 1), (1, 70, 37, True, 1),
                                                      (2, 128, 40, False, 2), (2, 64, 40, True, 2),
                                                      (3, 64, 40, False, 3), (3, 4, 512, True, 3)])
def test_two_phase_kernels_write_every_slot(fusion, nx, ny, walls, steps, prec):
    from paper_2302_04120_amd import lbm
    print_case(test="poison-phase", fusion=fusion, nx=nx, ny=ny, walls=walls, prec=prec)
    if walls:
        prm, ini, _ = WL.layered(nx=nx, ny=ny, seed=1, dx=5e-6, dt=2.5e-7, W_nodes=6)
    else:
        prm, ini, _ = WL.bubble(n=nx, ny=ny, radii=(min(nx, ny) // 4,), batch=1, seed=1)
    g = WL.rng(2)
    ini = dict(ini, ux=5e-3 * g.uniform(-1, 1, ini["phi"].shape),
               uy=5e-3 * g.uniform(-1, 1, ini["phi"].shape))

    def make():
        bc = (0, 0, lbm.BC_WALL, lbm.BC_WALL) if walls else (0, 0, 0, 0)
        L = lbm.Lattice("phase", nx, ny, prec=prec, bc=bc)
        L.set_step_fusion(fusion)
        L.set_graph_steps(0)
        L.set_params(prm)
        L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
        return L

    L, twin = make(), make()
    _poison_next(L, (19 if prec == "fp32" else 18) + 2)
    _check(L, twin, steps)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_d3q19_writes_every_slot(prec):
    from paper_2302_04120_amd import lbm
    print_case(test="poison-d3q19", prec=prec)
    nx, ny, nz = 70, 9, 5
    prm, ini = WL.box3d(nx, ny, nz, batch=1, seed=3, F=(40.0, -25.0, 15.0), mrt=True)

    def make():
        L = lbm.Lattice("d3q19", nx, ny, prec=prec, bc=(0, 0, 1, 1), nz=nz, bc_z=(1, 1))
        L.set_graph_steps(0)
        L.set_params(prm)
        L.init3d(ini["rho"], ini["ux"], ini["uy"], ini["uz"])
        return L

    L, twin = make(), make()
    _poison_next(L, 19)
    _check(L, twin, 1)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_phase3d_writes_every_slot(prec):
    from paper_2302_04120_amd import lbm
    print_case(test="poison-phase3d", prec=prec)
    nx, ny, nz = 70, 9, 5
    prm, ini = WL.bubble3d(n=nx, ny=ny, nz=nz, R_nodes=3.0, seed=1, u_noise=0.02)

    def make():
        L = lbm.Lattice("phase3d", nx, ny, prec=prec, bc=(1, 1, 0, 0), nz=nz, bc_z=(1, 1))
        L.set_graph_steps(0)
        L.set_params(prm)
        L.init3d(ini["p"], ini["ux"], ini["uy"], ini["uz"], ini["phi"])
        return L

    L, twin = make(), make()
    npl = (39 if prec == "fp32" else 38) + 3
    pb, plane = _pop_bytes(L, npl)
    # the phi plane sits at the end of the buffer, after the FP64 work areas
    _poison_next(L, npl, extra=[(L.bytes - (plane + 255) // 256 * 256, plane)])
    _check(L, twin, 1)


def test_the_poison_reaches_live_state_slots():
    """Control for the offsets used above: the same fill applied to the
    buffer that holds the current state (A, right after initialisation)
    turns the fields non-finite, so the poisoned ranges are live slots."""
    import torch
    from paper_2302_04120_amd import lbm
    print_case(test="poison-control")
    prm, ini, _ = WL.bubble(n=70, ny=37, radii=(9,), batch=1, seed=1)
    L = lbm.Lattice("phase", 70, 37, prec="fp32")
    L.set_graph_steps(0)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    torch.cuda.synchronize()
    pb, _ = _pop_bytes(L, 21)
    L.buf[:pb].fill_(255)
    torch.cuda.synchronize()
    L.step(1)
    m = L.macros(("phi",))
    assert not np.isfinite(m["phi"]).any()

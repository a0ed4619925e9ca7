"""The node-block state layout (two-phase D2Q9, heated channel, D3Q19, 3D
two-phase): every value of 64 consecutive nodes stored together, the last
block padded.  With a node count that is not a multiple of 64 the last block
is partial, and:

- a state blob holds exactly the N node values of each stored quantity (no
  padding), and a run resumed from it equals the uninterrupted run bit for
  bit;
- no kernel reads the padding: a run whose whole buffer was filled with NaN
  bytes before initialisation stays finite and equals a twin run on a fresh
  buffer bit for bit (a read of a padding slot would carry the NaN in)."""
import numpy as np
import pytest

from paper_2302_04120_amd import workloads as WL

from gpu_cases import print_case

pytestmark = pytest.mark.gpu


def _phase(prec, nx=37, ny=23, batch=2):
    from paper_2302_04120_amd import lbm
    # default 1702 nodes: 26 full blocks and 38 nodes
    prm, ini, _ = WL.bubble(n=nx, ny=ny, radii=(min(7, nx // 3, ny // 3),), batch=batch, seed=3)

    def make():
        L = lbm.Lattice("phase", nx, ny, batch=batch, prec=prec)
        L.set_params(prm)
        return L, lambda L: L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    return make, batch * nx * ny, (21 if prec == "fp32" else 20)


def _chan(prec):
    from paper_2302_04120_amd import lbm
    nx, ny = 150, 22  # 3300 nodes: 51 full blocks and 36 nodes
    prm, ini = WL.channel(nx=nx, ny=ny, dx=5e-5, tau_ratio=0.6, oscillating=True)

    def make():
        L = lbm.Lattice("channel", nx, ny, prec=prec,
                        bc=(lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL),
                        flow=True, thermal=True)
        L.set_params(prm)
        return L, lambda L: L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    return make, nx * ny, 14


def _d3(prec):
    from paper_2302_04120_amd import lbm
    nx, ny, nz = 10, 7, 5  # 350 nodes: 5 full blocks and 30 nodes
    prm, ini = WL.box3d(nx, ny, nz, seed=5)

    def make():
        L = lbm.Lattice("d3q19", nx, ny, prec=prec, nz=nz, bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
        L.set_params(prm)
        return L, lambda L: L.init3d(ini["rho"], ini["ux"], ini["uy"], ini["uz"])
    return make, nx * ny * nz, 19


def _p3(prec):
    from paper_2302_04120_amd import lbm
    nx, ny, nz = 12, 10, 7  # 840 nodes: 13 full blocks and 8 nodes
    props = {k: v for k, v in WL.TWO_PHASE_SYSTEMS["air_water_25C"].items()
             if k not in ("zeta_l", "zeta_g")}
    prm, ini = WL.bubble3d(n=nx, ny=ny, nz=nz, R_nodes=3.5, seed=6, **props)

    def make():
        L = lbm.Lattice("phase3d", nx, ny, prec=prec, nz=nz)
        L.set_params(prm)
        return L, lambda L: L.init3d(ini["p"], ini["ux"], ini["uy"], ini["uz"], ini["phi"])
    return make, nx * ny * nz, (42 if prec == "fp32" else 41)


CASES = {"phase": _phase, "channel": _chan, "d3q19": _d3, "phase3d": _p3,
         # 35 nodes: only a partial block; 128 nodes: two full blocks, no partial one
         "phase_35": lambda prec: _phase(prec, 7, 5, 1),
         "phase_128": lambda prec: _phase(prec, 16, 8, 1)}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("lattice", sorted(CASES))
def test_ragged_blocks_save_load_resume(lattice, prec):
    print_case(test="layout-resume", lattice=lattice, prec=prec)
    make, N, nvals = CASES[lattice](prec)
    a, init = make()
    init(a)
    a.step(9)
    blob = a.save_state()
    es = 4 if prec == "fp32" else 8
    header = len(a.save_state()) - nvals * N * es
    assert 0 < header <= 128  # the blob is a small header and the N values of each quantity
    a.step(11)
    b, _ = make()
    b.load_state(blob)
    assert b.t == 9
    b.step(11)
    assert a.save_state() == b.save_state()


PAD = 16448  # extra elements per value array of the library's buffer layout


@pytest.mark.parametrize("lattice", sorted(CASES))
def test_padding_never_read(lattice):
    import torch
    print_case(test="layout-padding", lattice=lattice)
    make, N, nvals = CASES[lattice]("fp32")
    poisoned, init = make()
    # the two state buffers lead the device buffer, each nvals arrays of
    # P = ceil64(N) + PAD elements rounded up to 256 bytes; what follows them
    # (the channel's wall-flux and inlet arrays) is left alone
    P = (N + 63) // 64 * 64 + PAD
    state_bytes = 2 * ((nvals * P * 4 + 255) // 256 * 256)
    torch.cuda.synchronize()
    poisoned.buf[:state_bytes].fill_(255)  # NaN bytes, the padding of both buffers included
    torch.cuda.synchronize()
    init(poisoned)
    clean, _ = make()
    init(clean)
    for n in (1, 2, 7):
        poisoned.step(n)
        clean.step(n)
        assert poisoned.reduce(("nonfinite",))["nonfinite"].sum() == 0
        assert poisoned.save_state() == clean.save_state()

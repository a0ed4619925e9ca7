"""The two-step (temporally blocked) channel kernel against the single-step
kernel.  Both evaluate the same per-node arithmetic (the shared collision and
boundary-value functions) in the same order, so a run of either must give the
same state to the last bit.  The cases cover the velocity inlet and pressure
outlet with the flux walls of the heated channel (Sec. 4.2), the differentially
heated cavity with the Boussinesq force (App. D), a buoyant channel with inlet
and outlet, the half channel under the symmetry plane, periodic x and y, one and several x-tiles (ragged and a multiple of
64), one and several row segments, a replica batch, BGK and MRT, FP32 and
FP64, the oscillating wall flux (a different modulation in each of the two
steps), a flux that varies along the wall, odd step counts (the last step
single) and graph replay."""
import numpy as np
import pytest

from paper_2302_04120_amd import workloads as WL

from gpu_cases import print_case

pytestmark = pytest.mark.gpu


def _case(nx, ny, seed, oscillating=False, **over):
    prm, ini = WL.channel(nx=nx, ny=ny, dx=5e-5, tau_ratio=0.7, oscillating=oscillating)
    g = WL.rng(seed)
    prm = dict(prm, **over)
    prm["flux"] = prm["q_s"] * g.uniform(0.5, 1.5, nx)
    ini = dict(ini)
    ini["ux"] = ini["ux"] + g.uniform(-1e-3, 1e-3, ini["ux"].shape)
    ini["uy"] = ini["uy"] + g.uniform(-1e-3, 1e-3, ini["uy"].shape)
    ini["T"] = ini["T"] + g.uniform(-0.5, 0.5, ini["T"].shape)
    return prm, ini


def _cavity_case(n, seed):
    """The App. D cavity (hot left wall, cold right wall, insulated top and
    bottom) with a perturbed start, so that the buoyancy acts everywhere."""
    prm, ini = WL.cavity(Ra=1e4, n=n)
    g = WL.rng(seed)
    ini = dict(ini)
    ini["T"] = ini["T"] + g.uniform(0.0, 40.0, ini["T"].shape)
    ini["ux"] = ini["ux"] + g.uniform(-1e-3, 1e-3, ini["ux"].shape)
    ini["uy"] = ini["uy"] + g.uniform(-1e-3, 1e-3, ini["uy"].shape)
    return prm, ini


def _state(prm, ini, nx, ny, bc, fusion, steps, prec="fp32", batch=1, graph_steps=0,
           thermal=True):
    from paper_2302_04120_amd import lbm
    L = lbm.Lattice("channel", nx, ny, prec=prec, bc=bc, batch=batch, thermal=thermal)
    L.set_graph_steps(graph_steps)
    L.set_params(prm)
    L.set_step_fusion(fusion)
    if batch > 1:
        ini = {k: np.broadcast_to(v, (batch,) + v.shape[-2:]).copy() for k, v in ini.items()}
    L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    for s in steps:
        L.step(s)
    blob = L.save_state()
    nonfinite = L.reduce(("nonfinite",))["nonfinite"].sum()
    L.close()
    return blob, nonfinite


def _bc(name):
    from paper_2302_04120_amd import lbm
    io = (lbm.BC_VEL_INLET, lbm.BC_P_OUTLET)
    walls = (lbm.BC_WALL, lbm.BC_WALL)
    xw = (lbm.BC_DIRICHLET, lbm.BC_DIRICHLET)
    return {"io_walls": io + walls, "px_walls": (0, 0) + walls, "periodic": (0, 0, 0, 0),
            "io_py": io + (0, 0), "cavity": xw + walls, "xw_py": xw + (0, 0),
            "io_symmetry": io + (lbm.BC_WALL, lbm.BC_SYMMETRY),
            "px_symmetry": (0, 0, lbm.BC_WALL, lbm.BC_SYMMETRY),
            "xw_symmetry": xw + (lbm.BC_WALL, lbm.BC_SYMMETRY)}[name]


CASES = [
    # name, nx, ny, bc, prec, batch, oscillating, overrides
    ("one_tile_osc", 200, 20, "io_walls", "fp32", 1, True, {}),
    ("tiles_ragged_segments", 600, 70, "io_walls", "fp32", 1, False, {}),
    ("tiles_aligned_segments", 512, 72, "io_walls", "fp32", 1, True, {}),
    ("bgk", 200, 20, "io_walls", "fp32", 1, False, {"flow_mrt": 0, "thermal_mrt": 0}),
    ("px_walls_force_wrapped", 128, 16, "px_walls", "fp32", 1, False, {"Fx": 50.0}),
    ("periodic_tiles_segments", 300, 70, "periodic", "fp32", 1, False, {"Fx": 50.0}),
    ("io_periodic_y", 256, 33, "io_py", "fp32", 1, False, {}),
    ("batch2", 128, 40, "px_walls", "fp32", 2, True, {"Fx": 50.0}),
    ("tiny_io", 3, 2, "io_walls", "fp32", 1, False, {}),
    ("tiny_periodic", 2, 2, "periodic", "fp32", 1, False, {"Fx": 50.0}),
    ("one_tile_osc_fp64", 200, 20, "io_walls", "fp64", 1, True, {}),
    ("tiles_ragged_segments_fp64", 600, 70, "io_walls", "fp64", 1, False, {}),
    ("tiles_aligned_fp64", 512, 40, "io_walls", "fp64", 1, False, {}),
    ("periodic_tiles_segments_fp64", 300, 70, "periodic", "fp64", 1, False, {"Fx": 50.0}),
    ("buoyant_io", 600, 70, "io_walls", "fp32", 1, False, {"beta_T": 3e-4, "gravity": (0.0, -9.81)}),
    ("buoyant_px_fp64", 300, 70, "px_walls", "fp64", 1, False,
     {"beta_T": 3e-4, "gravity": (2.0, -9.81)}),
    ("symmetry_plane", 600, 70, "io_symmetry", "fp32", 1, True, {}),
    ("symmetry_plane_fp64", 200, 20, "io_symmetry", "fp64", 1, False, {}),
    ("symmetry_periodic_x", 300, 40, "px_symmetry", "fp32", 1, False, {"Fx": 50.0}),
    ("batch3_io_aligned", 256, 40, "io_walls", "fp32", 3, True, {}),
]
CAVITY_CASES = [
    # name, n, bc, prec
    ("cavity_tiles_segments", 300, "cavity", "fp32"),
    ("cavity_aligned", 512, "cavity", "fp32"),
    ("cavity_fp64", 300, "cavity", "fp64"),
    ("end_walls_periodic_y", 260, "xw_py", "fp32"),
    ("cavity_tiny", 3, "cavity", "fp32"),
]


@pytest.mark.parametrize("name,nx,ny,bc,prec,batch,osc,over", CASES, ids=[c[0] for c in CASES])
def test_two_step_channel_kernel_bit_identical(name, nx, ny, bc, prec, batch, osc, over):
    print_case(test="chan-fusion", case=name, nx=nx, ny=ny, prec=prec, batch=batch)
    prm, ini = _case(nx, ny, seed=len(name), oscillating=osc, **over)
    steps = [7, 30]
    one, nf1 = _state(prm, ini, nx, ny, _bc(bc), 1, steps, prec=prec, batch=batch)
    two, nf2 = _state(prm, ini, nx, ny, _bc(bc), 2, steps, prec=prec, batch=batch)
    assert nf1 == 0 and nf2 == 0
    if one != two:
        a = np.frombuffer(one, np.uint8)
        b = np.frombuffer(two, np.uint8)
        pytest.fail("states differ in %d of %d bytes" % (int((a != b).sum()), a.size))


D2Q9_CASES = [
    # name, nx, ny, bc, prec, cavity, oscillating, overrides
    ("d2q9_io_walls_osc", 600, 70, "io_walls", "fp32", False, True, {}),
    ("d2q9_aligned", 512, 40, "io_walls", "fp32", False, False, {}),
    ("d2q9_half_channel", 600, 70, "io_symmetry", "fp32", False, True, {}),
    ("d2q9_half_channel_fp64", 200, 20, "io_symmetry", "fp64", False, False, {}),
    ("d2q9_periodic_buoyant", 300, 70, "periodic", "fp32", False, False,
     {"Fx": 50.0, "beta_T": 3e-4, "gravity": (0.0, -9.81)}),
    ("d2q9_io_periodic_y", 256, 33, "io_py", "fp32", False, False, {}),
    ("d2q9_tiny_io", 3, 2, "io_walls", "fp32", False, False, {}),
    ("d2q9_cavity", 300, 300, "cavity", "fp32", True, False, {}),
    ("d2q9_cavity_fp64", 130, 130, "cavity", "fp64", True, False, {}),
    ("d2q9_end_walls_symmetry", 260, 40, "xw_symmetry", "fp32", True, False, {}),
]


@pytest.mark.parametrize("name,nx,ny,bc,prec,cavity,osc,over", D2Q9_CASES,
                         ids=[c[0] for c in D2Q9_CASES])
def test_two_step_kernel_d2q9_thermal_bit_identical(name, nx, ny, bc, prec, cavity, osc, over):
    """The D2Q9 thermal set (Sec. 3, App. D): its diagonal links at the inlet
    (the mean inlet temperature of the two rows a link joins), the outlet
    extrapolation, the flux walls, the end walls and the symmetry plane."""
    print_case(test="chan-fusion-d2q9", case=name, nx=nx, ny=ny, prec=prec)
    if cavity:
        prm, ini = _cavity_case(nx, seed=len(name))
        if ny != nx:  # a cavity cut to ny rows: per-row inputs of ny entries
            ini = {k: v[:ny] for k, v in ini.items()}
            prm = dict(prm, inlet_u=np.zeros(ny), inlet_T=np.full(ny, prm["T_ref"]))
    else:
        prm, ini = _case(nx, ny, seed=len(name), oscillating=osc, **over)
    steps = [7, 30]
    one, nf1 = _state(prm, ini, nx, ny, _bc(bc), 1, steps, prec=prec, thermal="d2q9")
    two, nf2 = _state(prm, ini, nx, ny, _bc(bc), 2, steps, prec=prec, thermal="d2q9")
    assert nf1 == 0 and nf2 == 0
    if one != two:
        a = np.frombuffer(one, np.uint8)
        b = np.frombuffer(two, np.uint8)
        pytest.fail("states differ in %d of %d bytes" % (int((a != b).sum()), a.size))


@pytest.mark.parametrize("name,n,bc,prec", CAVITY_CASES, ids=[c[0] for c in CAVITY_CASES])
def test_two_step_kernel_cavity_bit_identical(name, n, bc, prec):
    print_case(test="chan-fusion-cavity", case=name, n=n, prec=prec)
    prm, ini = _cavity_case(n, seed=len(name))
    steps = [7, 30]
    one, nf1 = _state(prm, ini, n, n, _bc(bc), 1, steps, prec=prec)
    two, nf2 = _state(prm, ini, n, n, _bc(bc), 2, steps, prec=prec)
    assert nf1 == 0 and nf2 == 0
    if one != two:
        a = np.frombuffer(one, np.uint8)
        b = np.frombuffer(two, np.uint8)
        pytest.fail("states differ in %d of %d bytes" % (int((a != b).sum()), a.size))


def test_two_step_channel_kernel_under_graph_replay():
    """Captured runs of the two-step kernel (steady wall flux) replay to the
    same state as single steps launched one by one."""
    nx, ny = 600, 70
    print_case(test="chan-fusion-graph", nx=nx, ny=ny)
    prm, ini = _case(nx, ny, seed=3)
    one, _ = _state(prm, ini, nx, ny, _bc("io_walls"), 1, [41])
    two, _ = _state(prm, ini, nx, ny, _bc("io_walls"), 2, [41], graph_steps=8)
    assert one == two


@pytest.mark.parametrize("flow,thermal", [(True, False), (False, True)],
                         ids=["flow_only", "temperature_only"])
def test_two_step_channel_mode_rejected_where_not_covered(flow, thermal):
    """Mode 2 on a channel configuration the two-step kernel does not cover
    (flow alone, temperature alone) is refused once the parameters are set."""
    from paper_2302_04120_amd import lbm
    print_case(test="chan-fusion-unsupported", flow=flow, thermal=thermal)
    prm, ini = _case(64, 16, seed=1)
    L = lbm.Lattice("channel", 64, 16, bc=_bc("px_walls"), flow=flow, thermal=thermal)
    try:
        L.set_params(prm)
        with pytest.raises(lbm.LbmError) as ex:
            L.set_step_fusion(2)
        assert ex.value.status == lbm.LBM_E_UNSUPPORTED
        L.set_step_fusion(1)
    finally:
        L.close()


def test_two_step_channel_kernel_bench_size():
    """The roofline-sized channel of the bench (16384 x 2048, C2 physics) in
    the launch configuration the bench times (x-tiles on node-block-aligned
    rows, the segment model's row segments): the same state as single steps
    after two launches and a single step."""
    import hashlib

    from paper_2302_04120_amd import lbm
    nx, ny = 16384, 2048
    print_case(test="chan-fusion-bench-size", nx=nx, ny=ny)
    prm, ini = WL.channel(nx=nx, ny=ny)
    bc = _bc("io_walls")
    digests = []
    for fusion in (1, 2):
        L = lbm.Lattice("channel", nx, ny, bc=bc, thermal=True)
        L.set_graph_steps(0)
        L.set_params(prm)
        L.set_step_fusion(fusion)
        L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
        L.step(2)
        L.step(3)
        assert L.reduce(("nonfinite",))["nonfinite"].sum() == 0
        digests.append(hashlib.sha256(L.save_state()).hexdigest())
        L.close()
    assert digests[0] == digests[1]


def test_automatic_mode_on_a_large_channel():
    """8192 x 1024 (33 x-tiles, enough row segments to fill the GPU): the
    automatic kernel choice (the two-step kernel at this size) gives the same
    state as single steps."""
    import hashlib

    from paper_2302_04120_amd import lbm
    nx, ny = 8192, 1024
    print_case(test="chan-fusion-auto", nx=nx, ny=ny)
    prm, ini = _case(nx, ny, seed=9)
    digests = []
    for fusion in (1, 0):
        L = lbm.Lattice("channel", nx, ny, bc=_bc("io_walls"), thermal=True)
        L.set_graph_steps(0)
        L.set_params(prm)
        L.set_step_fusion(fusion)
        L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
        L.step(2)
        L.step(5)
        assert L.reduce(("nonfinite",))["nonfinite"].sum() == 0
        digests.append(hashlib.sha256(L.save_state()).hexdigest())
        L.close()
    assert digests[0] == digests[1]

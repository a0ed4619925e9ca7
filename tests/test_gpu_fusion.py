"""The two-step (temporally blocked) two-phase kernel against the single-step
kernel and the oracle.  Both kernels evaluate the same per-node arithmetic
in the same order, so a run of either must give the same state to the last
bit; the cases cover periodic and walled y, one and several 128-row
segments, rows in x-tiles (ragged, single, wrapped), odd step counts (the
last step single) and graph replay."""
import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

from gpu_cases import phase_pair, print_case, rel_err, u_abs_err, u_tol

pytestmark = pytest.mark.gpu


def _run(prm, ini, nx, ny, batch, prec, fusion, steps, walls, graph_steps=0):
    from paper_2302_04120_amd import lbm
    bc = (0, 0, lbm.BC_WALL, lbm.BC_WALL) if walls else (0, 0, 0, 0)
    L = lbm.Lattice("phase", nx, ny, batch=batch, prec=prec, bc=bc)
    L.set_step_fusion(fusion)
    L.set_graph_steps(graph_steps)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    for s in steps:
        L.step(s)
    return L


def _bubble_case(nx, ny, batch, seed):
    """Bubbles of radius 12-20 nodes in an nx x ny periodic cell."""
    prm, ini, _ = WL.bubble(n=nx, ny=ny, radii=(12, 16, 20), batch=batch, seed=seed)
    return prm, ini


def _layered_case(nx, ny):
    prm, ini, _ = WL.layered(nx=nx, ny=ny, seed=0, dx=5e-6, dt=1e-7, W_nodes=5.0)
    return prm, ini


CASES = [
    # nx, ny, batch, walls, steps
    (64, 64, 2, False, (7, 10)),      # one segment, odd call
    (128, 320, 1, False, (12,)),      # three 128-row segments, ragged last one
    (256, 256, 2, False, (6, 5)),     # two segments, the bench cell
    (64, 300, 1, True, (9, 8)),       # walls, ragged segments
    (192, 40, 1, True, (10,)),        # walls, one short segment
    # rows in x-tiles of 250 stored columns (nx not a multiple of 64 up to 256)
    (300, 70, 1, False, (9, 8)),      # two tiles, the second one ragged
    (250, 40, 2, False, (6,)),        # exactly one tile
    (251, 33, 1, False, (5,)),        # one tile and one column
    (100, 64, 1, False, (4,)),        # one tile holding the row 2.5 times
    (7, 20, 1, False, (3, 4)),        # a very narrow row
    (520, 300, 1, True, (9, 8)),      # walls, three tiles, ragged segments
    (600, 130, 2, False, (5,)),       # three tiles, one segment per replica
]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("nx,ny,batch,walls,steps", CASES)
def test_two_step_kernel_bit_identical(nx, ny, batch, walls, steps, prec):
    print_case(test="tb2-bits", nx=nx, ny=ny, batch=batch, walls=walls, prec=prec)
    if walls:
        prm, ini = _layered_case(nx, ny)
        batch = 1
    else:
        prm, ini = _bubble_case(nx, ny, batch, seed=nx + ny)
    one = _run(prm, ini, nx, ny, batch, prec, 1, steps, walls)
    two = _run(prm, ini, nx, ny, batch, prec, 2, steps, walls)
    s1, s2 = one.save_state(), two.save_state()
    if s1 != s2:
        m1, m2 = one.macros(("phi", "p", "ux")), two.macros(("phi", "p", "ux"))
        diffs = {k: float(np.abs(m1[k] - m2[k]).max()) for k in m1}
        raise AssertionError("two-step state differs from single-step: %s" % diffs)
    assert one.t == two.t == sum(steps)
    red = two.reduce(("phase", "nonfinite"))
    assert red["nonfinite"].sum() == 0


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_two_step_kernel_with_graph_replay(prec):
    """Graph replay of two-step launches: the graph makes an odd number of
    buffer swaps per replay (graph_steps / 2 = 3)."""
    prm, ini = _bubble_case(128, 128, 2, seed=5)
    print_case(test="tb2-graph", prec=prec)
    ref = _run(prm, ini, 128, 128, 2, prec, 1, (), False)
    gr = _run(prm, ini, 128, 128, 2, prec, 2, (), False, graph_steps=6)
    for rep, n in enumerate((13, 12, 25)):
        ref.step(n)
        gr.step(n)
        assert ref.save_state() == gr.save_state(), rep


def test_two_step_kernel_against_oracle():
    """Direct parity of the two-step path with the FP64 oracle (FP32
    deviation storage, 20 steps, one bubble in a 256 x 128 cell)."""
    prm, ini = _bubble_case(256, 128, 1, seed=11)
    print_case(test="tb2-oracle")
    g, o, L, _ = phase_pair(prm, ini, 256, 128, 20, "fp32", fusion=2)
    scale_p = max(float(np.abs(o["p"]).max()), prm["sigma"] / prm["W"])
    assert rel_err(g["phi"], o["phi"], scale=1.0) < 1e-5
    assert rel_err(g["p"], o["p"], scale=scale_p) < 1e-5
    assert u_abs_err(g, o) < u_tol(prm, o)


def test_fusion_validation():
    from paper_2302_04120_amd import lbm
    prm, ini = _bubble_case(96, 64, 1, seed=0)
    L = lbm.Lattice("phase", 96, 64, prec="fp32")
    L.set_step_fusion(2)  # nx not a multiple of 64: rows in x-tiles
    for bad in (4, -1):
        with pytest.raises(lbm.LbmError) as e:
            L.set_step_fusion(bad)
        assert e.value.status == lbm.LBM_E_ARG
    L.set_step_fusion(1)


@pytest.mark.timeout(300)
def test_bench_size_two_step_sampled_against_oracle():
    """The benchmark's own launch configuration: 1024 replicas of the 256 x 256
    bubble cell (67 M nodes, FP32, two-step kernel), 20 steps.  Sampled
    replicas (the first, a middle and the last, which sit in different
    segments and XCD bands) against the FP64 oracle run one by one; every
    replica's phi sum conserved and no non-finite population anywhere."""
    from paper_2302_04120_amd import lbm
    batch, n, steps = 1024, 256, 20
    prm, ini, _ = WL.bubble(n=n, batch=batch, seed=0)
    print_case(test="tb2-bench-size", batch=batch, steps=steps)
    L = lbm.Lattice("phase", n, n, batch=batch, prec="fp32")
    L.set_step_fusion(2)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    m0 = L.reduce(("phase",))["phase"]
    L.step(steps)
    red = L.reduce(("phase", "nonfinite"))
    assert red["nonfinite"].sum() == 0
    assert (np.abs(red["phase"] - m0) / m0).max() < 1e-13
    m = L.macros(("phi", "p", "ux"))
    for b in (0, 513, 1023):
        o = O.Phase(n, n, prm)
        o.init(ini["phi"][b], ini["p"][b], ini["ux"][b], ini["uy"][b])
        o.step(steps)
        mo = o.macros()
        scale_p = max(float(np.abs(mo["p"]).max()), prm["sigma"] / prm["W"])
        e = (rel_err(m["phi"][b], mo["phi"], scale=1.0), rel_err(m["p"][b], mo["p"], scale=scale_p),
             rel_err(m["ux"][b], mo["ux"]))
        du = u_abs_err({"ux": m["ux"][b]}, mo)
        print("replica %d: phi %.2e p %.2e ux %.2e (|du| %.2e m/s)" % (b, *e, du), flush=True)
        assert e[0] < 1e-5 and e[1] < 1e-5 and du < u_tol(prm, mo)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("nx,ny,walls", [(4, 300, True), (8, 200, True), (16, 70, True),
                                         (32, 45, False)])
def test_narrow_replica_tiles_against_oracle(nx, ny, walls, prec, tol):
    """Replicas narrower than 64 nodes (the C4 shape is 4 x 512) run on tiles
    of nx x 256/nx nodes (FP32; nx x 512/nx in FP64): every lane holds a node and ragged rows cross tile
    edges.  Parity with the oracle for three replicas, 20 steps: the layered
    channel between walls, and a bubble for the periodic case (a layered
    profile is not periodic in y)."""
    from paper_2302_04120_amd import lbm
    batch, steps = 3, 20
    if walls:
        prm, ini, _ = WL.layered(nx=nx, ny=ny, seed=nx, dx=5e-6, dt=2.5e-7, W_nodes=6, batch=batch)
    else:
        prm, ini, _ = WL.bubble(n=nx, ny=ny, radii=(nx // 3,), batch=batch, seed=nx)
    g = WL.rng(nx + 1)
    # velocities well above the FP32 resolution of the gas momentum (the z_i
    # carry the pressure scale, so a 1e-3 m/s field sits at ~1e-4 relative)
    ini = dict(ini, ux=5e-3 * g.uniform(-1, 1, ini["phi"].shape),
               uy=5e-3 * g.uniform(-1, 1, ini["phi"].shape))
    print_case(test="narrow-tiles", nx=nx, ny=ny, walls=walls, prec=prec)
    bc = (0, 0, lbm.BC_WALL, lbm.BC_WALL) if walls else (0, 0, 0, 0)
    L = lbm.Lattice("phase", nx, ny, batch=batch, prec=prec, bc=bc)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    L.step(steps)
    m = L.macros(("phi", "p", "ux"))
    for b in range(batch):
        o = O.Phase(nx, ny, prm, bc_y="walls" if walls else "periodic")
        o.init(ini["phi"][b], ini["p"][b], ini["ux"][b], ini["uy"][b])
        o.step(steps)
        mo = o.macros()
        scale_p = max(float(np.abs(mo["p"]).max()), prm["sigma"] / prm["W"])
        e = (rel_err(m["phi"][b], mo["phi"], scale=1.0), rel_err(m["p"][b], mo["p"], scale=scale_p),
             rel_err(m["ux"][b], mo["ux"]))
        print("replica %d: phi %.2e p %.2e ux %.2e" % (b, *e), flush=True)
        assert e[0] < tol and e[1] < tol
        if prec == "fp64":
            assert e[2] < tol
        else:
            assert u_abs_err({"ux": m["ux"][b]}, mo) < u_tol(prm, mo)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec,batch", [("fp32", 512), ("fp64", 256)])
def test_whole_replica_segments_bit_identical(prec, batch):
    """Batches large enough to fill the GPU's resident workgroups on their
    own run the two-step kernel on whole 256-row replicas (no segments); the
    state after 4 steps (both paths then hold it in buffer A) equals that of
    single-step launches node by node, compared on the device."""
    import torch
    from paper_2302_04120_amd import lbm
    n = 256
    prm, ini, _ = WL.bubble(n=n, batch=batch, seed=7)
    print_case(test="tb2-whole-replicas", prec=prec, batch=batch)
    runs = []
    for fusion in (1, 2):
        L = lbm.Lattice("phase", n, n, batch=batch, prec=prec)
        L.set_step_fusion(fusion)
        L.set_params(prm)
        L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
        L.step(4)
        torch.cuda.synchronize()
        runs.append(L)
    # the state buffer starts with the node blocks of the current state: all
    # planes of 64 consecutive nodes together, N a multiple of 64 here
    N = batch * n * n
    assert N % 64 == 0
    planes = 21 if prec == "fp32" else 20
    dt = torch.float32 if prec == "fp32" else torch.float64
    es = 4 if prec == "fp32" else 8
    views = [L.buf[:planes * N * es].view(dt) for L in runs]
    assert torch.equal(views[0], views[1])
    assert runs[1].reduce(("nonfinite",))["nonfinite"].sum() == 0

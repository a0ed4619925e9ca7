"""The many-steps-per-launch two-phase kernel (step fusion mode 3) against
single-step launches.  One resident workgroup per tile steps its tile and
waits only for the step counters of the tiles it exchanges data with, so a
missing wait shows up as a state that differs from the single-step kernel's;
both evaluate the same per-node arithmetic in the same order, so the states
must agree to the last bit.  The cases cover the narrow C4 replica (4 x 512
between walls), periodic square cells, several replicas, ragged tiles with a
one-node tail (where every tile waits for all tiles of its replica), odd step
counts, several calls in a row (the counters carry over) and a state
reloaded from a blob."""
import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

from gpu_cases import print_case, rel_err, u_abs_err, u_tol

pytestmark = pytest.mark.gpu


def _lattice(prm, ini, nx, ny, batch, prec, walls, fusion, graph_steps=0):
    from paper_2302_04120_amd import lbm
    bc = (0, 0, lbm.BC_WALL, lbm.BC_WALL) if walls else (0, 0, 0, 0)
    L = lbm.Lattice("phase", nx, ny, batch=batch, prec=prec, bc=bc)
    L.set_step_fusion(fusion)
    L.set_graph_steps(graph_steps)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    return L


def _case(nx, ny, batch, walls, seed):
    if walls:
        prm, ini, _ = WL.layered(nx=nx, ny=ny, seed=seed, dx=5e-6, dt=2.5e-7, W_nodes=6,
                                 batch=batch)
    else:
        prm, ini, _ = WL.bubble(n=nx, ny=ny, radii=(max(2, min(nx, ny) // 4),), batch=batch,
                                seed=seed)
    g = WL.rng(seed + 1)
    ini = dict(ini, ux=5e-3 * g.uniform(-1, 1, ini["phi"].shape),
               uy=5e-3 * g.uniform(-1, 1, ini["phi"].shape))
    return prm, ini


CASES = [
    # nx, ny, batch, walls, step calls      tiles of the kernel
    (4, 512, 1, True, (101,)),              # 16 of 4 x 32: the C4 replica
    (4, 512, 3, True, (50, 51)),            # 12 of 4 x 128
    (8, 100, 1, True, (47,)),               # 7 of 8 x 16, ragged y
    (32, 33, 1, False, (40,)),              # 9 of 32 x 4, one-row tail
    (64, 64, 2, False, (33, 40)),           # 16 of 64 x 8, one column per replica
    (192, 24, 1, False, (31,)),             # 9 of 64 x 8, periodic 3 x 3 neighbourhoods
    (256, 32, 1, False, (40, 9)),           # 16 of 64 x 8, tiles two apart do not wait
    (70, 17, 2, False, (37,)),              # 12 of 64 x 8, one-column and one-row tails
    (130, 26, 1, True, (25, 1, 24)),        # 12 of 64 x 8, tails of 2 nodes, walls
    (16, 70, 2, False, (45,)),              # 10 of 16 x 16, ragged y
    (100, 8, 1, False, (64,)),              # 4 of 64 x 4
]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("nx,ny,batch,walls,calls", CASES)
def test_many_steps_kernel_bit_identical(nx, ny, batch, walls, calls, prec):
    print_case(test="persist-bits", nx=nx, ny=ny, batch=batch, walls=walls, prec=prec)
    prm, ini = _case(nx, ny, batch, walls, seed=nx + ny)
    one = _lattice(prm, ini, nx, ny, batch, prec, walls, 1)
    many = _lattice(prm, ini, nx, ny, batch, prec, walls, 3)
    for n in calls:
        one.step(n)
        many.step(n)
        assert one.t == many.t
        s1, s3 = one.save_state(), many.save_state()
        if s1 != s3:
            m1, m3 = one.macros(("phi", "p", "ux")), many.macros(("phi", "p", "ux"))
            diffs = {k: float(np.abs(m1[k] - m3[k]).max()) for k in m1}
            raise AssertionError("after %d steps: many-steps state differs: %s" % (one.t, diffs))
    assert many.reduce(("nonfinite",))["nonfinite"].sum() == 0


def test_many_steps_kernel_after_reload_and_mode_switch():
    """Counters restart with a reloaded state; switching modes between calls
    (single-step, graph replay, many-steps) keeps the trajectory."""
    nx, ny = 64, 40
    prm, ini = _case(nx, ny, 1, False, seed=9)
    print_case(test="persist-reload")
    ref = _lattice(prm, ini, nx, ny, 1, "fp32", False, 1)
    ref.step(300)
    L = _lattice(prm, ini, nx, ny, 1, "fp32", False, 3)
    L.step(77)
    blob = L.save_state()
    L.step(500)  # counters well past the reloaded state's
    L.load_state(blob)
    L.step(23)
    L.set_step_fusion(1)
    L.set_graph_steps(16)
    L.step(100)
    L.set_step_fusion(3)
    L.step(100)
    assert L.t == ref.t == 300
    assert L.save_state() == ref.save_state()


def test_many_steps_kernel_against_oracle():
    """Direct parity with the FP64 oracle: the C4 replica, FP32 deviation
    storage, 40 steps in one launch."""
    nx, ny, steps = 4, 512, 40
    prm, ini = _case(nx, ny, 1, True, seed=3)
    print_case(test="persist-oracle")
    L = _lattice(prm, ini, nx, ny, 1, "fp32", True, 3)
    L.step(steps)
    m = {k: v[0] for k, v in L.macros(("phi", "p", "ux")).items()}
    o = O.Phase(nx, ny, prm, bc_y="walls")
    o.init(ini["phi"][0], ini["p"][0], ini["ux"][0], ini["uy"][0])
    o.step(steps)
    mo = o.macros()
    scale_p = max(float(np.abs(mo["p"]).max()), prm["sigma"] / prm["W"])
    assert rel_err(m["phi"], mo["phi"], scale=1.0) < 1e-5
    assert rel_err(m["p"], mo["p"], scale=scale_p) < 1e-5
    assert u_abs_err(m, mo) < u_tol(prm, mo)


def test_many_steps_mode_validation():
    from paper_2302_04120_amd import lbm
    print_case(test="persist-validation")
    L = lbm.Lattice("phase", 96, 200, prec="fp32")  # 2 x 25 tiles
    with pytest.raises(lbm.LbmError):
        L.set_step_fusion(3)
    with pytest.raises(lbm.LbmError):
        L.set_step_fusion(4)
    L2 = lbm.Lattice("phase", 4, 512, batch=5, prec="fp32")  # 5 x 4 tiles of 4 x 128
    with pytest.raises(lbm.LbmError):
        L2.set_step_fusion(3)
    lbm.Lattice("phase", 4, 512, batch=4, prec="fp32").set_step_fusion(3)  # 16 tiles


def test_many_steps_error_word_is_reported_and_the_state_dropped():
    """The host-side error path of the many-steps mode, forced from the host:
    the error word that a timed-out wait would set is written into the
    context's buffer before the call (it follows the 16 step counters in the
    buffer's last 256 bytes for this lattice).  The kernel's waits see it and
    leave (or the run completes), lbm_step reports LBM_E_DEVICE and drops the
    state, and a new initialisation clears the word and steps normally."""
    import torch
    from paper_2302_04120_amd import lbm
    nx, ny = 64, 40
    prm, ini = _case(nx, ny, 1, False, seed=12)
    print_case(test="persist-error-word")
    L = _lattice(prm, ini, nx, ny, 1, "fp32", False, 3)
    torch.cuda.synchronize()
    L.buf[-256 + 64:-256 + 68] = torch.tensor([1, 0, 0, 0], dtype=torch.uint8, device=L.buf.device)
    torch.cuda.synchronize()
    with pytest.raises(lbm.LbmError) as e:
        L.step(20)
    assert e.value.status == lbm.LBM_E_DEVICE
    with pytest.raises(lbm.LbmError) as e:
        L.step(1)
    assert e.value.status == lbm.LBM_E_STATE
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    L.step(20)
    ref = _lattice(prm, ini, nx, ny, 1, "fp32", False, 1)
    ref.step(20)
    assert L.save_state() == ref.save_state()

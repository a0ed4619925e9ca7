"""The two-step kernel on a single wide domain: the 8192 x 8192 periodic
bubble array (32 x 32 different 256^2 bubble cells in one domain), whose
rows the kernel takes in x-tiles of 250 stored columns.

Parity at this size uses the domain of dependence: one step of the model
reads the populations of the nearest neighbours (streaming) and phi of the
nearest neighbours (the stencils), so after s steps a node depends only on
the initial state within 2 s nodes.  A cell's interior farther than 2 s + 2
nodes from its edges therefore evolves exactly as in the oracle's run of that
cell alone (periodic on its own), and is compared node by node."""
import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

from gpu_cases import print_case, rel_err, u_abs_err, u_tol

pytestmark = pytest.mark.gpu

CELLS, N = 32, 256


@pytest.mark.timeout(600)
def test_bubble_array_8192_two_step_matches_oracle_cells():
    from paper_2302_04120_amd import lbm
    steps = 20
    prm, ini, _ = WL.bubble_array(CELLS, N, seed=0)
    L = lbm.Lattice("phase", CELLS * N, CELLS * N, prec="fp32")
    L.set_step_fusion(0)  # the library's own choice: the tiled two-step kernel here
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    m0 = L.reduce(("phase",))["phase"][0]
    print_case(test="wide-8192", steps=steps)
    L.step(steps)
    red = L.reduce(("phase", "nonfinite"))
    assert red["nonfinite"][0] == 0
    assert abs(red["phase"][0] - m0) < 1e-13 * m0
    g = {k: v[0] for k, v in L.macros(("phi", "p", "ux", "uy")).items()}
    L.close()
    _, cells, _ = WL.bubble(n=N, batch=CELLS * CELLS, seed=0)
    margin = 2 * steps + 2
    inner = slice(margin, N - margin)
    for (i, j) in ((0, 0), (5, 17), (31, 31), (16, 0)):
        b = i * CELLS + j
        o = O.Phase(N, N, prm)
        o.init(cells["phi"][b], cells["p"][b], cells["ux"][b], cells["uy"][b])
        o.step(steps)
        mo = {k: v[inner, inner] for k, v in o.macros().items()}
        gc = {k: v[i * N:(i + 1) * N, j * N:(j + 1) * N][inner, inner] for k, v in g.items()}
        scale_p = max(float(np.abs(mo["p"]).max()), prm["sigma"] / prm["W"])
        e = {"phi": rel_err(gc["phi"], mo["phi"], scale=1.0),
             "p": rel_err(gc["p"], mo["p"], scale=scale_p)}
        du = u_abs_err(gc, mo)
        print("cell", (i, j), e, "|du| %.3e bound %.3e" % (du, u_tol(prm, mo)), flush=True)
        assert e["phi"] < 1e-5 and e["p"] < 1e-5, (i, j, e)
        assert du < u_tol(prm, mo), (i, j, du)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_wide_domain_two_step_bit_identical_to_single_steps(prec):
    """8192 x 512 rows of bubble cells (33 x-tiles, four 128-row segments),
    with walls: the tiled two-step kernel and single-step launches end in the
    same state to the last bit, over an odd step count."""
    from paper_2302_04120_amd import lbm
    prm, ini, _ = WL.bubble_array(2, 256, seed=3)
    ini = {k: np.tile(v, (1, 1, 16))[:, :512, :8192] for k, v in ini.items()}
    print_case(test="wide-bits", prec=prec)
    states = []
    for fusion in (1, 2):
        L = lbm.Lattice("phase", 8192, 512, prec=prec, bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
        L.set_step_fusion(fusion)
        L.set_params(prm)
        L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
        L.step(9)
        states.append(L.save_state())
        L.close()
    assert states[0] == states[1]

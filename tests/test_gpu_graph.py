"""Graph replay of lbm_step: a run of steps enqueued as one captured HIP graph
must give bit-identical states to the same steps launched one by one.  Each
case replays the graphs several times, with reductions, macro read-backs and
stream synchronisations between the replays, and compares every replay."""
import numpy as np
import pytest

from paper_2302_04120_amd import workloads as WL

from gpu_cases import print_case

pytestmark = pytest.mark.gpu


def _phase(prm, ini, n, batch, prec, graph_steps):
    from paper_2302_04120_amd import lbm
    L = lbm.Lattice("phase", n, n, batch=batch, prec=prec)
    L.set_graph_steps(graph_steps)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    return L


def _channel(prm, ini, nx, ny, prec, graph_steps):
    from paper_2302_04120_amd import lbm
    L = lbm.Lattice("channel", nx, ny, prec=prec,
                    bc=(lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL),
                    flow=True, thermal=True)
    L.set_graph_steps(graph_steps)
    L.set_params(prm)
    L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    return L


def _same(a, b):
    """Bit-identical saved states (populations, parity, step count)."""
    sa, sb = a.save_state(), b.save_state()
    return len(sa) == len(sb) and sa == sb


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_phase_graph_replay_bit_identical(prec):
    prm, ini, _ = WL.bubble(n=64, radii=(12, 16), batch=2, seed=3)
    print_case(test="graph-phase", prec=prec)
    eager = _phase(prm, ini, 64, 2, prec, 0)
    graph = _phase(prm, ini, 64, 2, prec, 8)
    # 21 steps: two replays of 8 plus 5 single launches, so the parity of
    # the state changes between calls and both captured graphs get used
    for rep in range(4):
        eager.step(21)
        graph.step(21)
        r_e = eager.reduce(("phase", "mass", "nonfinite"))
        r_g = graph.reduce(("phase", "mass", "nonfinite"))
        assert r_g["nonfinite"].sum() == 0
        for k in r_e:
            assert np.array_equal(r_e[k], r_g[k]), (rep, k)
        m_e, m_g = eager.macros(("p", "phi", "ux")), graph.macros(("p", "phi", "ux"))
        for k in m_e:
            assert np.array_equal(m_e[k], m_g[k]), (rep, k)
        assert _same(eager, graph), rep
        assert eager.t == graph.t == 21 * (rep + 1)


def test_channel_graph_replay_bit_identical_and_new_params():
    prm, ini = WL.channel(nx=96, ny=24)
    print_case(test="graph-channel")
    eager = _channel(prm, ini, 96, 24, "fp32", 0)
    graph = _channel(prm, ini, 96, 24, "fp32", 16)
    for rep in range(3):
        eager.step(50)
        graph.step(50)
        assert _same(eager, graph), rep
        ne, ng = eager.nusselt(48), graph.nusselt(48)
        for a, b in zip(ne, ng):
            assert np.array_equal(np.asarray(a), np.asarray(b)), rep
    # new parameters must not replay the stale captured arguments
    prm2, _ = WL.channel(nx=96, ny=24, q_s=2 * prm["q_s"])
    eager.set_params(prm2)
    graph.set_params(prm2)
    for rep in range(2):
        eager.step(40)
        graph.step(40)
        assert _same(eager, graph), ("after set_params", rep)


def test_oscillating_flux_is_never_replayed():
    """The oscillating wall flux changes with the step count, so lbm_step
    launches it step by step even with graph replay enabled."""
    prm, ini = WL.channel(nx=96, ny=24, oscillating=True)
    eager = _channel(prm, ini, 96, 24, "fp64", 0)
    graph = _channel(prm, ini, 96, 24, "fp64", 8)
    eager.step(64)
    graph.step(64)
    assert _same(eager, graph)


def test_graph_steps_validation():
    from paper_2302_04120_amd import lbm
    prm, ini, _ = WL.bubble(n=64, radii=(12, 16), batch=1, seed=0)
    L = _phase(prm, ini, 64, 1, "fp32", 0)
    for bad in (-2, 3, 4098):
        with pytest.raises(lbm.LbmError):
            L.set_graph_steps(bad)
    L.set_graph_steps(4)
    L.step(9)
    assert L.t == 9


@pytest.mark.parametrize("fusion", [1, 3])
def test_caller_captured_steps_replay(fusion):
    """A caller that captures lbm_step(n) on its own stream (torch's graph
    capture) and replays the graph gets n more steps per replay: the capture
    takes single-step launches whatever the step fusion mode (the many-steps
    kernel synchronises and so is not captured), and every replay matches
    eager single-step launches to the bit.  n is even, so each replay starts
    from the buffer the capture started in."""
    import torch
    from paper_2302_04120_amd import lbm
    nx, ny, n = 64, 48, 8
    prm, ini, _ = WL.bubble(n=nx, ny=ny, radii=(10,), batch=1, seed=4)
    print_case(test="caller-capture", fusion=fusion)
    s = torch.cuda.Stream()

    def make(stream, mode):
        L = lbm.Lattice("phase", nx, ny, batch=1, prec="fp32", stream=stream)
        L.set_step_fusion(mode)
        L.set_params(prm)
        L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
        return L

    cap = make(s, fusion)
    ref = make(None, 1)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cap.step(n)
    assert cap.t == n  # counted once, at capture
    fields = ("phi", "p", "ux", "uy")
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        ref.step(n)
        a, b = cap.macros(fields), ref.macros(fields)
        for k in fields:
            assert np.array_equal(a[k], b[k]), (rep, k)
        assert ref.reduce(("nonfinite",))["nonfinite"].sum() == 0

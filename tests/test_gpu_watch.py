"""Failure detection inside lbm_step (the periodic non-finite check and the
step it reports) and the FP32 forcing guard of lbm_set_params_SI."""
import struct
import warnings

import numpy as np
import pytest

from paper_2302_04120_amd import workloads as WL

from gpu_cases import print_case

pytestmark = pytest.mark.gpu

HDR = 4 + 4 + 6 * 4 + 8 + 8 + 8 + 8  # state blob header bytes before the first value


def _channel(every, graph=0):
    from paper_2302_04120_amd import lbm
    L = lbm.Lattice("channel", 40, 16, prec="fp32", flow=True)
    L.set_graph_steps(graph)
    L.set_nonfinite_check(every)
    L.set_params(dict(dx=1e-5, dt=1e-4, rho_ref=1000.0, nu=1e-6, Fx=50.0))
    L.init(np.full((16, 40), 1000.0))
    return L


def _plant_nan(L, t_blob=None):
    blob = bytearray(L.save_state())
    blob[HDR:HDR + 4] = struct.pack("<f", float("nan"))
    L.load_state(bytes(blob))


def test_no_report_on_a_finite_run_and_the_check_changes_nothing():
    print_case(test="watch-finite")
    a, b = _channel(100, graph=64), _channel(0, graph=64)
    for L in (a, b):
        L.step(700)
    assert a.first_nonfinite_step() == -1 and b.first_nonfinite_step() == -1
    assert a.save_state() == b.save_state()  # the check only reads


@pytest.mark.parametrize("every,steps,expect", [(50, 120, 50), (64, 200, 64), (0, 120, -1)])
def test_planted_nan_is_reported_with_its_step(every, steps, expect):
    from paper_2302_04120_amd import lbm
    print_case(test="watch-nan", every=every)
    L = _channel(every)
    _plant_nan(L)
    L.step(steps)
    assert L.first_nonfinite_step() == expect
    with pytest.raises(lbm.LbmError) as e:
        L.reduce()
    assert e.value.status == lbm.LBM_E_NONFINITE
    if expect > 0:
        assert "step %d" % expect in str(e.value)


def test_check_counts_steps_from_the_loaded_state():
    """A state saved at step 130 and loaded with a NaN: the next multiple of
    the interval (150) is the first check."""
    print_case(test="watch-offset")
    L = _channel(50)
    L.step(130)
    _plant_nan(L)
    assert L.t == 130
    L.step(7)
    assert L.first_nonfinite_step() == -1
    L.step(30)
    assert L.first_nonfinite_step() == 150


def test_check_in_the_two_phase_fused_and_many_steps_modes():
    print_case(test="watch-phase")
    from paper_2302_04120_amd import lbm
    prm, ini, _ = WL.layered(nx=4, ny=512, seed=0, dx=5e-6, dt=2.5e-7, W_nodes=6)
    for fusion in (2, 3):
        L = lbm.Lattice("phase", 4, 512, prec="fp32", bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
        L.set_step_fusion(fusion)
        L.set_nonfinite_check(40)
        L.set_params(prm)
        L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
        L.step(100)
        assert L.first_nonfinite_step() == -1
        _plant_nan(L)
        L.step(25)
        assert L.first_nonfinite_step() == 120
        L.close()


def test_fp32_forcing_guard():
    """The layered channel at the paper's finest grid: the slow liquids (water
    at 100 and 80 C) are flagged in FP32, the faster ones (25 C) are not, and
    neither FP64 nor FP32 storage with FP64 arithmetic is flagged."""
    from paper_2302_04120_amd import lbm
    print_case(test="fp32-guard")
    got = {}
    for system in ("sat_water_100C", "sat_water_80C", "sat_water_25C", "air_water_25C"):
        props = {k: v for k, v in WL.TWO_PHASE_SYSTEMS[system].items()
                 if k in ("rho_l", "rho_g", "nu_l", "nu_g", "sigma")}
        prm, _, _ = WL.layered(nx=4, ny=512, seed=0, dx=1.25e-6, dt=1.25e-8, W_nodes=20.0, **props)
        for prec in ("fp32", "fp64", "fp32_arith64"):
            L = lbm.Lattice("phase", 4, 512, prec=prec, bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
            with warnings.catch_warnings(record=True) as w:
                warnings.simplefilter("always")
                st = L.set_params(prm)
            got[(system, prec)] = st
            assert (st == lbm.LBM_W_FP32_FORCING) == bool(w)
            L.close()
    assert got[("sat_water_100C", "fp32")] == lbm.LBM_W_FP32_FORCING
    assert got[("sat_water_80C", "fp32")] == lbm.LBM_W_FP32_FORCING
    assert got[("sat_water_25C", "fp32")] == lbm.LBM_OK
    assert got[("air_water_25C", "fp32")] == lbm.LBM_OK
    for system in ("sat_water_100C", "sat_water_80C"):
        assert got[(system, "fp64")] == lbm.LBM_OK
        assert got[(system, "fp32_arith64")] == lbm.LBM_OK


def test_check_interval_validation():
    from paper_2302_04120_amd import lbm
    L = _channel(10)
    with pytest.raises(lbm.LbmError) as e:
        L.set_nonfinite_check(-1)
    assert e.value.status == lbm.LBM_E_ARG


def test_mach_warning_on_inlet_and_initial_velocity():
    """LBM_W_MACH: an inlet profile or an initial velocity faster than 0.3 dx/dt
    is reported (bit set, RuntimeWarning) while the call still takes effect;
    the C2 channel's own speeds are far below and report nothing."""
    from paper_2302_04120_amd import lbm
    print_case(test="mach-warning")
    nx, ny = 64, 16
    prm, ini = WL.channel(nx=nx, ny=ny)
    c = prm["dx"] / prm["dt"]
    bc = (lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL)

    def quiet(fn, *a):
        with warnings.catch_warnings(record=True) as w:
            warnings.simplefilter("always")
            st = fn(*a)
        return st, [str(x.message) for x in w]

    L = lbm.Lattice("channel", nx, ny, prec="fp32", bc=bc, flow=True, thermal=True)
    st, w = quiet(L.set_params, prm)
    assert st == lbm.LBM_OK and not w
    st, w = quiet(L.init, ini["rho"], ini["ux"], ini["uy"], ini["T"])
    assert st == lbm.LBM_OK and not w
    fast = dict(prm, inlet_u=prm["inlet_u"] * (0.35 * c / prm["inlet_u"].max()))
    st, w = quiet(L.set_params, fast)
    print("inlet:", w, flush=True)
    assert st == lbm.LBM_W_MACH and len(w) == 1 and "inlet profile" in w[0]
    L.close()

    # the initial velocity of a two-phase box (all liquid, so that no interface
    # force enters the velocity read back): at 0.29 c nothing, at 0.31 c the
    # warning, and the fields are set either way
    prm, _, _ = WL.bubble(n=64, radii=(14,), batch=1, seed=0)
    c = prm["dx"] / prm["dt"]
    zero, one = np.zeros((64, 64)), np.ones((64, 64))
    for frac, want in ((0.29, lbm.LBM_OK), (0.31, lbm.LBM_W_MACH)):
        L = lbm.Lattice("phase", 64, 64, prec="fp64")
        L.set_params(prm)
        ux = np.full((64, 64), 0.1 * c)
        ux[5, 7] = -frac * c
        st, w = quiet(L.init, zero, ux, zero, None, one)
        print(frac, st, w, flush=True)
        assert st == want and bool(w) == (want != lbm.LBM_OK)
        got = L.macros(("ux",))["ux"][0]
        assert np.abs(got - ux).max() < 1e-9 * c
        L.close()

    # the 3D initial velocity, with the speed in z only
    L = lbm.Lattice("d3q19", 8, 8, nz=8, prec="fp32")
    L.set_params(dict(dx=1e-3, dt=1e-3, rho_ref=1.0, nu=1e-4))
    uz = np.zeros((8, 8, 8))
    uz[3, 4, 5] = 0.5
    st, w = quiet(L.init3d, np.ones((8, 8, 8)), None, None, uz)
    assert st == lbm.LBM_W_MACH and "initial velocity" in w[0]
    L.close()

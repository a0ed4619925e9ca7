"""Physics of the configurations at their full sizes on the GPU, against what
the paper fixes (closed forms and its printed accuracy levels), and FP32
deviation storage against FP64 on the same runs."""
import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

from gpu_cases import FP32_TOL, fixed_point_tol, print_case

pytestmark = pytest.mark.gpu


def _chan(prm, ini, nx, ny, prec):
    from paper_2302_04120_amd import lbm
    L = lbm.Lattice("channel", nx, ny, prec=prec,
                    bc=(lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL),
                    flow=True, thermal=True)
    L.set_params(prm)
    L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    return L


@pytest.mark.parametrize("oscillating", [False, True])
def test_c2_channel_developed_nusselt_fp32_vs_fp64(oscillating):
    """C2 (800 x 40, developed inlet, uniform wall flux 1e4 W/m^2), 50 000 steps:
    the local Nu over the downstream half is the developed 140/17 = 8.235
    (Sec. 4.2; the paper's own LBM got 8.15, 1 %), and the FP32-deviation run
    matches the FP64 run.  The last 20 columns are left out of the pointwise
    check: the zero-gradient thermal outlet bends the profile there (Nu drops
    to ~7.9 in the final ~10 columns).  The oscillating variant
    q0 (1 + 0.5 sin wt) has no closed form; only its FP32/FP64 agreement is
    checked.

    FP32 against FP64: velocity and density to the 1e-5 target (measured
    1.6e-6 and 1.5e-6).  Temperature to 1e-4, and below
    gpu_cases.fixed_point_tol of its slowest mode: the cross-section mean of
    T is not restored by diffusion between flux walls but flushed out in
    L / u_m, u_m dt / L = 3.6e-5 per step, which lets the rounded run settle
    up to 1.6e-3 of max |T - T_ref| away (measured 2.9e-5)."""
    nx, ny, steps = 800, 40, 50000
    prm, ini = WL.channel(oscillating=oscillating)
    print_case(test="c2", oscillating=oscillating, dt=prm["dt"])
    out = {}
    for prec in ("fp64", "fp32"):
        L = _chan(prm, ini, nx, ny, prec)
        L.step(steps)
        out[prec] = (L.macros(), L.nusselt(nx // 2))
    m64, (Tb, Tw, Nu, nm, tout) = out["fp64"]
    m32, (Tb32, _, Nu32, nm32, tout32) = out["fp32"]
    errs = {"T": np.abs(m32["T"] - m64["T"]).max() / np.abs(m64["T"] - prm["T_ref"]).max(),
            "ux": np.abs(m32["ux"] - m64["ux"]).max() / np.abs(m64["ux"]).max(),
            "uy": np.abs(m32["uy"] - m64["uy"]).max() / np.abs(m64["ux"]).max(),
            "rho": np.abs(m32["rho"] - m64["rho"]).max() / np.abs(m64["rho"] - prm["rho_ref"]).max()}
    H, Lc = ny * prm["dx"], nx * prm["dx"]
    alpha = prm["alpha"]
    t_tol = fixed_point_tol(prm["dt"] * min(alpha * (np.pi / H) ** 2, prm["u_m"] / Lc))
    print("Nu mean (x >= L/2) fp64 %.5f fp32 %.5f; T_out %.6f / %.6f; FP32-vs-FP64 %s; "
          "T bound %.2e" % (nm, nm32, tout, tout32, errs, t_tol), flush=True)
    for k in ("ux", "uy", "rho"):
        assert errs[k] < FP32_TOL, (k, errs[k])
    assert errs["T"] < min(1e-4, t_tol)
    assert abs(nm32 - nm) < 1e-3 * nm
    if not oscillating:
        core = slice(nx // 2, nx - 20)
        print("Nu over x in [L/2, L - 20 dx]: min %.4f max %.4f mean %.4f" %
              (Nu[core].min(), Nu[core].max(), Nu[core].mean()), flush=True)
        assert np.abs(Nu[core] - 140 / 17).max() < 0.02 * 140 / 17
        assert abs(Nu[core].mean() - 140 / 17) < 0.01 * 140 / 17
        # energy balance: T_b rises by 2 q'' / (rho c_p u_m H) per metre
        xs = np.arange(nx)[core] * prm["dx"]
        slope = np.polyfit(xs, Tb[core], 1)[0]
        assert slope == pytest.approx(2 * prm["q_s"] / (prm["rho_cp"] * prm["u_m"] * prm["H"]),
                                      rel=0.03)


def test_c3_bubble_laplace_law_and_mass():
    """C3 (256 x 256 periodic, 4 radii 20/30/40/50 nodes, density ratio 43 290,
    viscosity ratio 471) in FP32 deviation storage, run until the pressure
    jump has settled (120 000 steps = 12 ms; the largest bubble's jump still
    moves by 20 % between 20 000 and 40 000 steps and by < 0.2 % after
    120 000): the jump follows Laplace's law sigma / R (the paper reports
    4.3-5.1 % for its 5-node interface; accepted within 8 % per radius for the
    4-node one used here), the density profile follows Eq. density_prof
    within the paper's 0.25-0.46 % order (accepted < 1 %), the
    order-parameter sum is conserved to FP64 reduction rounding, and the FP32
    jump matches the FP64 one."""
    from paper_2302_04120_amd import lbm
    n, steps = 256, 120000
    prm, ini, cen = WL.bubble(n=n, batch=4, seed=0)
    print_case(test="c3", steps=steps)
    res = {}
    for prec in ("fp32", "fp64"):
        L = lbm.Lattice("phase", n, n, batch=4, prec=prec)
        L.set_params(prm)
        L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
        m0 = L.reduce(("phase",))["phase"]
        L.step(steps)
        m1 = L.reduce(("phase",))["phase"]
        res[prec] = (L.macros(), np.abs(m1 - m0) / m0)
    x = WL.node_centres(n, prm["dx"])
    X, Y = np.meshgrid(x, x)
    m32, drift32 = res["fp32"]
    m64, drift64 = res["fp64"]
    print("phase-mass drift fp32", drift32, "fp64", drift64, flush=True)
    assert drift32.max() < 1e-13
    for b, (xc, yc, R) in enumerate(cen):
        r = np.hypot(X - xc, Y - yc)
        inside, outside = r < R - 2 * prm["W"], r > R + 2 * prm["W"]
        dps = {}
        for prec, (m, _) in res.items():
            dps[prec] = m["p"][b][inside].mean() - m["p"][b][outside].mean()
        rho_a = prm["rho_g"] + WL.tanh_profile(r - R, prm["W"]) * (prm["rho_l"] - prm["rho_g"])
        e2 = O.e2(rho_a, m32["rho"][b])
        lap = 100 * abs(dps["fp32"] - prm["sigma"] / R) / (prm["sigma"] / R)
        print("R = %d dx: dP fp32 %.3f fp64 %.3f sigma/R %.3f (%.2f %%), density E2 %.3f %%" %
              (round(R / prm["dx"]), dps["fp32"], dps["fp64"], prm["sigma"] / R, lap, e2), flush=True)
        assert lap < 8.0
        assert e2 < 1.0
        assert dps["fp32"] == pytest.approx(dps["fp64"], rel=1e-3)


def _layered(prm, ini, nx, ny, prec):
    from paper_2302_04120_amd import lbm
    L = lbm.Lattice("phase", nx, ny, prec=prec, bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    return L


def test_c4_layered_startup_stokes_layer():
    """C4 at its full size (4 x 512, dx = 1.25 um, dt = 12.5 ns, W = 25 um,
    density ratio 43 290) from rest, 200 000 steps (2.5 ms).  Below the
    interface the liquid obeys u_t = nu_l u_yy + F/rho_l with no slip at the
    wall, whose solution from rest is
        u = (F t / rho_l) [1 - 4 i^2erfc(eta)],  eta = y / (2 sqrt(nu_l t))
    (Stokes' first problem with a body force).  Checked on nodes 10-90, where
    the interface, 166+ nodes away, has not reached (its influence there is
    below 0.3 %); FP32 deviation storage against FP64 on the whole field, and
    the order-parameter sum conserved to FP64 reduction rounding."""
    from scipy.special import erfc
    nx, ny, steps = 4, 512, 200000
    prm, ini, offs = WL.layered(nx=nx, ny=ny, seed=0)
    print_case(test="c4-startup", dt=prm["dt"], W=prm["W"], Fx=prm["Fx"])
    res = {}
    for prec in ("fp64", "fp32"):
        L = _layered(prm, ini, nx, ny, prec)
        m0 = L.reduce(("phase",))["phase"]
        L.step(steps)
        red = L.reduce(("phase", "nonfinite"))
        assert red["nonfinite"].sum() == 0
        res[prec] = (L.macros(("ux", "uy", "phi")), abs(red["phase"][0] - m0[0]) / m0[0])
    t = steps * prm["dt"]
    a = prm["Fx"] / prm["rho_l"]
    y = WL.node_centres(ny, prm["dx"])
    eta = y / (2 * np.sqrt(prm["nu_l"] * t))
    i2 = ((1 + 2 * eta ** 2) * erfc(eta) - 2 / np.sqrt(np.pi) * eta * np.exp(-eta ** 2)) / 4
    u_ref = a * t * (1 - 4 * i2)
    m64, d64 = res["fp64"]
    m32, d32 = res["fp32"]
    u = m32["ux"][0, :, 0]
    core = slice(10, 91)
    err = np.abs(u[core] - u_ref[core]).max() / (a * t)
    print("liquid: max |u - u_ref| / (F t / rho_l) = %.3e on nodes 10-90; u(50) %.5e ref %.5e; "
          "phase drift fp32 %.2e fp64 %.2e" % (err, u[50], u_ref[50], d32, d64), flush=True)
    assert err < 0.01
    # FP32 against FP64.  The liquid moves at u/c ~ 2e-8 here: its momentum
    # rho u / c ~ 2e-5 rides on z-populations that also carry p / c_s^2, so
    # FP32 storage resolves it to ~1e-6 of itself per step, and the rounding
    # accumulates over 2e5 steps to ~1e-3 (5e-3 accepted).  The gas velocity,
    # resolved only to eps_32 (p / c_s^2) / rho_g, is held to 3e-4 of the
    # largest (gas) speed.
    liq = m64["phi"] > 0.5
    scale = np.abs(m64["ux"]).max()
    e_liq = np.abs(m32["ux"] - m64["ux"])[liq].max() / np.abs(m64["ux"][liq]).max()
    e_all = np.abs(m32["ux"] - m64["ux"]).max() / scale
    print("FP32 vs FP64: liquid %.2e, whole field %.2e" % (e_liq, e_all), flush=True)
    assert e_liq < 5e-3
    assert e_all < 3e-4
    # u_y is only the decaying acoustic residue of the start from rest (the
    # weakly compressible gas; FP64 2e5 steps: 7e-7 m/s, 8e-4 of max u_x)
    assert np.abs(m64["uy"]).max() < 2e-3 * scale
    assert np.abs(m32["uy"] - m64["uy"]).max() < 5e-3 * scale
    assert d32 < 1e-13


def _golden_layered():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "layered_coarse_oracle.json")) as f:
        return json.load(f)


@pytest.mark.timeout(300)
def test_c4_layered_coarse_grid_steady_against_oracle_and_paper():
    """The layered flow of C4 on the coarsest grid of the paper's grid study
    (Sec. 4.4: dx = 5 um, dt = 0.1 us, W = 25 um = 5 dx; 128 nodes across, so
    H = 0.64 mm where the paper's channel is 0.5 mm),
    run from rest to steady state (3e6 steps, 6.5 liquid decay times) in
    FP32 deviation storage.  The steady profile matches the FP64 oracle's
    (stored by tests/golden/make_layered_coarse.py) node by node, and its E2
    against the diffuse-interface quadrature of Eq. NSE_for_layered_poiseuille
    is the oracle's, 17.0 %: the paper reports 16.1 % for this grid (its worst
    system, saturated water at 25 C, i.e. the density and viscosity ratios of
    this case), falling to 3.8 % and 1.6 % as dx and dt are halved.

    Node-by-node bound: gpu_cases.fixed_point_tol of the slowest viscous mode,
    nu_l dt (pi / H)^2 = 2.1e-6 per step, i.e. 2.8e-2 of max u: over the
    millions of steps to steady state the FP32 run settles on a fixed point of
    its rounded step, and this is how far such a point can sit from the exact
    one.  (Measured 1.1e-3; the E2 check below holds the two runs to 0.05
    points, i.e. 0.3 % of E2.)"""
    from layered_ref import diffuse_profile
    g = _golden_layered()
    nx, ny = g["nx"], g["ny"]
    prm, ini, offs = WL.layered(nx=nx, ny=ny, seed=g["seed"], dx=g["dx"], dt=g["dt"],
                                W_nodes=g["W_nodes"])
    print_case(test="c4-coarse", steps=g["steps"])
    L = _layered(prm, ini, nx, ny, "fp32")
    L.step(g["steps"])
    m = L.macros(("ux", "phi"))
    u, phi = m["ux"][0, :, 0], m["phi"][0, :, 0]
    u_o = np.asarray(g["ux"])
    y = WL.node_centres(ny, prm["dx"])
    e2 = O.e2(diffuse_profile(y, phi, prm, ny * prm["dx"]), u)
    pt = np.abs(u - u_o).max() / np.abs(u_o).max()
    H = ny * prm["dx"]
    tol = fixed_point_tol(min(prm["nu_l"], prm["nu_g"]) * prm["dt"] * (np.pi / H) ** 2)
    print("coarse grid: E2 vs diffuse quadrature %.3f %% (oracle %.3f %%, paper 16.132 %%); "
          "max |u - u_oracle| / max u %.2e (bound %.2e)" % (e2, g["E2_vs_diffuse_percent"], pt, tol),
          flush=True)
    assert pt < tol
    assert abs(e2 - g["E2_vs_diffuse_percent"]) < 0.05

"""Shared runners for the GPU parity tests: the same seeded inputs go to the
HIP path (through the C-ABI binding) and to the FP64 oracle, and the fields
are compared element by element.

Parity metric (per field): max |X_gpu - X_oracle| / max |X_oracle - X_ref|,
X_ref = rho_ref for density, T_ref for temperature, 0 otherwise.  The FP32
bound 1e-5 is the accuracy target for macroscopic fields; the FP64 path must
agree to rounding (1e-10 after hundreds of steps).
"""
import numpy as np

import oracle as O

FP32_TOL = 1e-5
FP64_TOL = 1e-10
EPS = {"fp32": 2.0 ** -23, "fp64": 2.0 ** -52}  # spacing of the numbers at 1
EPS32 = EPS["fp32"]
# FP32 and FP64 rounding units of the stored pressure populations allowed in
# the velocity of the lightest phase (see u_tol)
U_RES_UNITS = 4.0
# relative velocity floor of u_tol: the accuracy target in FP32, rounding in
# FP64 (the pressure populations of the two-phase model carry ~1e3 times the
# gas momentum, so FP64 velocities agree to ~1e-13 of max |u|)
U_REL = {"fp32": 1e-5, "fp64": 1e-12}


def u_resolution(prm, p_orc, prec="fp32"):
    """Velocity that one rounding unit of the stored pressure populations
    stands for in the lightest phase.  The z_i carry p / c_s^2 (kg/m^3) while
    the momentum they hold is rho u, and u = c sum(e_i z_i) / rho (Eq. u_Liang),
    so storage in precision prec resolves u only to EPS c max(|p|, sigma / W) /
    c_s^2 / rho_g -- in FP32, in the gas of the bubble case (rho_g = 0.0231
    kg/m^3), about 1e-3 of the spurious currents."""
    c = prm["dx"] / prm["dt"]
    p_scale = max(float(np.max(np.abs(p_orc))), prm.get("sigma", 0.0) / prm["W"])
    return EPS[prec] * c * p_scale / (c * c / 3.0) / min(prm["rho_g"], prm["rho_l"])


def u_fp32_resolution(prm, p_orc):
    return u_resolution(prm, p_orc, "fp32")


def u_tol(prm, o, prec="fp32"):
    """Absolute velocity bound of the two-phase parity tests: U_REL[prec] of
    max |u|, or U_RES_UNITS rounding units of the stored pressure populations
    in the lightest phase, whichever is larger.  o: the oracle's macros."""
    keys = [k for k in ("ux", "uy", "uz") if k in o]
    umax = max(float(np.max(np.abs(o[k]))) for k in keys)
    return max(U_REL[prec] * umax, U_RES_UNITS * u_resolution(prm, o["p"], prec))


def u_fp32_tol(prm, o):
    return u_tol(prm, o, "fp32")


def u_abs_err(g, o):
    """max |u_gpu - u_oracle| over the velocity components present in both."""
    keys = [k for k in ("ux", "uy", "uz") if k in o and k in g]
    return max(float(np.max(np.abs(np.asarray(g[k]) - o[k]))) for k in keys)


def accumulated_tol(steps, prec="fp32"):
    """A priori bound for a field of unit scale after `steps` steps whose
    every step adds at most one rounding unit of the storage precision:
    steps * EPS (the run's own FP32 error budget, used where a uniform flow
    of 5-10 % of c makes each step's rounding of the growing momentum and of
    the moving interface add up)."""
    return steps * EPS[prec]


def fixed_point_tol(rate_per_step, prec="fp32"):
    """A priori bound, relative to a field's scale, on how far a run that has
    settled (or is settling) in precision prec can sit from the exact one:
    each step rounds the field by about one rounding unit EPS / 2 of its scale,
    while the slowest mode is pulled back toward the exact solution by the
    fraction rate_per_step per step (viscous: nu dt k^2 with k = pi / H;
    flushed through a channel: u_m dt / L), so a fixed point of the rounded
    map lies within (EPS / 2) / rate_per_step of the exact one."""
    return 0.5 * EPS[prec] / rate_per_step


def rel_err(gpu, orc, ref=0.0, scale=None):
    """max |gpu - orc| / max |orc - ref|; ``scale`` overrides the denominator
    when the field's deviation range is smaller than the size of the stored
    populations that carry it (see the per-test comments)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    orc = np.asarray(orc, dtype=np.float64)
    if scale is None:
        scale = np.max(np.abs(orc - ref))
    if scale == 0:
        return float(np.max(np.abs(gpu - orc)))
    return float(np.max(np.abs(gpu - orc)) / scale)


def density_scale(rho_orc, rho_ref, u_orc, c):
    """Scale of the deviation populations of the momentum field: they hold
    w_i (rho - rho_ref) + w_i rho 3 e_i.u/c, so FP32 storage resolves density to
    a fraction of max(|rho - rho_ref|, 3 rho_ref |u|/c), not of |rho - rho_ref|
    alone; in FP64 the oracle's own rounding of rho ~ rho_ref sets the floor."""
    return max(float(np.max(np.abs(rho_orc - rho_ref))),
               3.0 * rho_ref * float(np.max(np.abs(u_orc))) / c)


def print_case(**kw):
    print("CASE " + " ".join("%s=%s" % kv for kv in kw.items()), flush=True)


def channel_pair(prm, ini, nx, ny, steps, prec, bc_x="inlet_outlet", bc_y="walls", thermal=True,
                 flow=True, batch=1, fusion=0):
    """Run the channel on the GPU and in the oracle; returns (gpu macros of
    replica 0, oracle macros, lattice object, oracle object).  fusion 2 steps
    the GPU side in pairs with the two-step kernel."""
    from paper_2302_04120_amd import lbm
    bcx = (lbm.BC_VEL_INLET, lbm.BC_P_OUTLET) if bc_x == "inlet_outlet" else (0, 0)
    bcy = (lbm.BC_WALL, lbm.BC_WALL) if bc_y == "walls" else (0, 0)
    L = lbm.Lattice("channel", nx, ny, batch=batch, prec=prec, bc=bcx + bcy, flow=flow,
                    thermal=thermal)
    L.set_params(prm)
    L.set_step_fusion(fusion)
    L.init(ini["rho"], ini["ux"], ini["uy"], ini.get("T") if thermal else None)
    L.step(steps)
    g = L.macros()
    o = O.Chan(nx, ny, prm, bc_x=bc_x, bc_y=bc_y, flow=flow, thermal=thermal)
    o.init(ini["rho"], ini["ux"], ini["uy"], ini.get("T") if thermal else None)
    o.step(steps)
    return {k: v[0] for k, v in g.items()}, o.macros(), L, o


def phase_pair(prm, ini, nx, ny, steps, prec, bc_y="periodic", replica=0, batch=None, fusion=0):
    from paper_2302_04120_amd import lbm
    phi = ini["phi"]
    if batch is None:
        batch = phi.shape[0]
    bcy = (lbm.BC_WALL, lbm.BC_WALL) if bc_y == "walls" else (0, 0)
    L = lbm.Lattice("phase", nx, ny, batch=batch, prec=prec, bc=(0, 0) + bcy)
    L.set_step_fusion(fusion)
    L.set_params(prm)
    L.init(ini["p"][:batch], ini["ux"][:batch], ini["uy"][:batch], None, phi[:batch])
    L.step(steps)
    g = L.macros()
    o = O.Phase(nx, ny, prm, bc_y=bc_y)
    o.init(phi[replica], ini["p"][replica], ini["ux"][replica], ini["uy"][replica])
    o.step(steps)
    return {k: v[replica] for k, v in g.items()}, o.macros(), L, o

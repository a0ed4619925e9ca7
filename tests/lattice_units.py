"""Conversion of SI inputs to the conventional lattice units of Sec. 3.

Test helper for the dimensional == conventional pin: C_x = dx, C_t = dt and a
density scale C_rho (the bubble case of Sec. 4.3 uses C_rho = 1 kg/m^3); for
temperature T~ = (T - T_ref) / C_T with C_T = 1 K.  Every other scale follows
from the SI units of the quantity.
"""
import numpy as np


def scales(dx, dt, C_rho=1.0):
    Cu = dx / dt
    return dict(x=dx, t=dt, rho=C_rho, u=Cu, nu=dx * dx / dt, omega=1.0 / dt,
                force=C_rho * dx / (dt * dt),         # N/m^3 = kg m^-2 s^-2
                pressure=C_rho * Cu * Cu,             # Pa
                sigma=C_rho * dx ** 3 / (dt * dt),    # N/m = kg s^-2
                grad=1.0 / dx)


def chan_to_lattice(prm):
    """SI channel parameters -> lattice parameters (dx = dt = 1)."""
    dx, dt = prm["dx"], prm["dt"]
    S = scales(dx, dt)
    out = dict(prm)
    out.update(dx=1.0, dt=1.0, rho_ref=prm.get("rho_ref", 1.0) / S["rho"],
               nu=prm.get("nu", 1e-6) / S["nu"], alpha=prm.get("alpha", 1e-7) / S["nu"],
               omega_e=prm.get("omega_e", 1.0 / dt) * dt, omega_eps=prm.get("omega_eps", 1.0 / dt) * dt,
               Fx=prm.get("Fx", 0.0) / S["force"], Fy=prm.get("Fy", 0.0) / S["force"],
               qvol=prm.get("qvol", 0.0) / prm.get("rho_cp", 1.0) * dt, T_ref=0.0,
               rho_cp=1.0,
               flux=np.asarray(prm.get("flux", 0.0)) * dt / (dx * prm.get("rho_cp", 1.0)),
               flux_omega=prm.get("flux_omega", 0.0) * dt,
               inlet_u=np.asarray(prm.get("inlet_u", 0.0)) / S["u"],
               inlet_T=np.asarray(prm.get("inlet_T", prm.get("T_ref", 0.0))) - prm.get("T_ref", 0.0))
    return out


def phase_to_lattice(prm, C_rho=1.0):
    dx, dt = prm["dx"], prm["dt"]
    S = scales(dx, dt, C_rho)
    out = dict(prm)
    out.update(dx=1.0, dt=1.0, rho_l=prm["rho_l"] / C_rho, rho_g=prm["rho_g"] / C_rho,
               nu_l=prm["nu_l"] / S["nu"], nu_g=prm["nu_g"] / S["nu"],
               zeta_l=prm["zeta_l"] / (C_rho * S["nu"]), zeta_g=prm["zeta_g"] / (C_rho * S["nu"]),
               sigma=prm["sigma"] / S["sigma"], W=prm["W"] / dx, M=prm["M"] / S["nu"],
               Fx=prm.get("Fx", 0.0) / S["force"], Fy=prm.get("Fy", 0.0) / S["force"],
               normal_eps=prm.get("normal_eps", 1e-12 / dx) * dx)
    return out

"""Reference profiles of the layered two-phase Poiseuille flow (Sec. 4.4).

The steady x-momentum balance d/dy (zeta du/dy) + F_x = 0 (Eq.
NSE_for_layered_poiseuille) with no slip at y = 0 and y = H integrates in
closed form for any viscosity profile zeta(y):
    u(y) = int_0^y (C - F s) / zeta(s) ds,  C = F int_0^H s/zeta / int_0^H 1/zeta.
With zeta taken from the simulated order parameter (zeta = zeta_g + phi
(zeta_l - zeta_g), Sec. 4.4) this is the diffuse-interface reference the paper
compares against; with a step in zeta it is the sharp-interface solution.
Evaluated by the trapezoidal rule on a fine grid."""
import numpy as np


def _integrate(y, H, zeta_of_s, F, n=200001):
    s = np.linspace(0.0, H, n)
    zeta = zeta_of_s(s)
    Cc = F * np.trapezoid(s / zeta, s) / np.trapezoid(1.0 / zeta, s)
    integ = (Cc - F * s) / zeta
    U = np.concatenate([[0.0], np.cumsum(0.5 * (integ[1:] + integ[:-1]) * np.diff(s))])
    return np.interp(y, s, U)


def diffuse_profile(y, phi, prm, H):
    """u(y) for zeta interpolated linearly in the node values of phi."""
    zl, zg = prm["zeta_l"], prm["zeta_g"]
    return _integrate(y, H, lambda s: zg + np.interp(s, y, phi) * (zl - zg), prm["Fx"])


def sharp_profile(y, y_int, prm, H):
    """u(y) for liquid (zeta_l) below y_int and gas (zeta_g) above."""
    zl, zg = prm["zeta_l"], prm["zeta_g"]
    return _integrate(y, H, lambda s: np.where(s < y_int, zl, zg), prm["Fx"])

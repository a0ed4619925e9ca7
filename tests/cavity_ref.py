"""Nusselt numbers of the App. D cavity from the macroscopic fields.

Mean over the cavity: steady energy conservation makes the horizontal heat
flow through every vertical line the same, Q = int (u T - alpha dT/dx) dy;
averaging Q over the width turns the conduction part into alpha (T_h - T_c)
(the wall temperatures are held exactly), so
    Nu = Q / (alpha (T_h - T_c)) = 1 + L <u T> / (alpha (T_h - T_c)),
with <.> the mean over all nodes.  Hot wall: Nu_0 = -(L / dT) <dT/dx> at the
wall x = 0 (halfway between the first node and its image), the derivative
from the second-order one-sided formula (-8 T_w + 9 T_1 - T_2) / (3 dx) on the
wall value and the first two node centres."""
import numpy as np


def nusselt_mean(ux, T, prm):
    dT = prm["Th"] - prm["Tc"]
    return 1.0 + prm["L"] * float(np.mean(ux * T)) / (prm["alpha"] * dT)


def nusselt_hot_wall(T, prm):
    dT = prm["Th"] - prm["Tc"]
    T1, T2 = T[:, 0], T[:, 1]
    dTdx = (-8.0 * prm["Th"] + 9.0 * T1 - T2) / (3.0 * prm["dx"])
    return float(np.mean(-dTdx)) * prm["L"] / dT

"""torch.autograd bridge to the discrete adjoint of the heated channel.

``ChannelAdjoint`` holds one channel lattice (D2Q9 flow + D2Q5 temperature,
inlet/outlet, flux walls) and its initial fields.  ``ChannelAdjoint.J(flux,
tau)`` returns the objective J = w_tout T_out + w_nu mean Nu after ``nsteps``
steps as a torch scalar whose backward runs the library's hand-written
adjoint (lbm_grad): gradients with respect to the wall-flux profile
(W/m^2, one value per column) and to (tau, tau_T) (s).  Forward and backward
both run in the HIP kernels behind the C ABI; this module only marshals.
"""
import numpy as np

from . import lbm


def _make_function():
    import torch

    class ChannelObjective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, flux, tau, problem):
            J = problem._forward(flux.detach().cpu().double().numpy(),
                                 tau.detach().cpu().double().numpy())
            ctx.problem = problem
            ctx.flux_meta = (flux.dtype, flux.device)
            ctx.tau_meta = (tau.dtype, tau.device)
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            gq, gt = ctx.problem.L.grad(float(gJ))
            dq = torch.as_tensor(gq, dtype=ctx.flux_meta[0], device=ctx.flux_meta[1])
            dt = torch.as_tensor(gt, dtype=ctx.tau_meta[0], device=ctx.tau_meta[1])
            return dq, dt, None

    return ChannelObjective


_FN = None


class ChannelAdjoint:
    """prm/ini: SI parameters and initial fields of the channel (see
    workloads.channel / workloads.adjoint_channel)."""

    def __init__(self, prm, ini, nx, ny, nsteps, ckpt_every, x_dev=None, w_tout=1.0, w_nu=1.0,
                 prec="fp32", device="cuda:0"):
        self.prm = dict(prm)
        self.ini = ini
        self.nx, self.ny = nx, ny
        self.nsteps, self.ckpt = nsteps, ckpt_every
        self.x_dev = nx // 2 if x_dev is None else x_dev
        self.w = (w_tout, w_nu)
        self.L = lbm.Lattice("channel", nx, ny, prec=prec,
                             bc=(lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL),
                             flow=True, thermal=True, device=device)
        dx, dt = prm["dx"], prm["dt"]
        self.cs2 = (dx / dt) ** 2 / 3.0

    def tau_of(self):
        """Current (tau, tau_T) implied by nu and alpha."""
        dt = self.prm["dt"]
        return np.array([self.prm["nu"] / self.cs2 + dt / 2, self.prm["alpha"] / self.cs2 + dt / 2])

    def _forward(self, flux, tau):
        dt = self.prm["dt"]
        prm = dict(self.prm, flux=flux, nu=(tau[0] - dt / 2) * self.cs2,
                   alpha=(tau[1] - dt / 2) * self.cs2)
        self.L.set_params(prm)
        self.L.init(self.ini["rho"], self.ini["ux"], self.ini["uy"], self.ini["T"])
        return self.L.record(self.nsteps, self.ckpt, self.x_dev, *self.w)

    def J(self, flux, tau):
        global _FN
        if _FN is None:
            _FN = _make_function()
        return _FN.apply(flux, tau, self)

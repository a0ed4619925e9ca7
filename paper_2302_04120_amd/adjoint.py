"""torch.autograd bridge to the discrete adjoint of the heated channel.

``ChannelAdjoint`` holds one channel lattice (D2Q9 flow + D2Q5 temperature,
inlet/outlet, flux walls) and its initial fields.  ``ChannelAdjoint.J(flux,
tau)`` returns the objective J = w_tout T_out + w_nu mean Nu after ``nsteps``
steps as a torch scalar whose backward runs the library's hand-written
adjoint (lbm_grad): gradients with respect to the wall-flux profile
(W/m^2, one value per column) and to (tau, tau_T) (s).  Forward and backward
both run in the HIP kernels behind the C ABI; this module only marshals (the
relaxation times go to the library as they are, through the tau and tau_T
parameters).

The library keeps the checkpoints of the last recorded forward run only.
Each forward run gets a generation number; a backward through an older
graph node re-records that node's own forward run (flux and tau saved with
it) before differentiating, so every backward returns the gradient at its own
inputs, whatever ran in between.
"""
import numpy as np

from . import lbm


def _make_function():
    import torch

    class ChannelObjective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, flux, tau, problem):
            q = flux.detach().cpu().double().numpy().copy()
            t = tau.detach().cpu().double().numpy().copy()
            J = problem._forward(q, t)
            ctx.problem = problem
            ctx.generation = problem.generation
            ctx.inputs = (q, t)
            ctx.flux_meta = (flux.dtype, flux.device)
            ctx.tau_meta = (tau.dtype, tau.device)
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            prob = ctx.problem
            if prob.generation != ctx.generation:
                # another forward run replaced the library's checkpoints
                prob._forward(*ctx.inputs)
            gq, gt = prob.L.grad(float(gJ))
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
        self.generation = 0
        self.L = lbm.Lattice("channel", nx, ny, prec=prec,
                             bc=(lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL),
                             flow=True, thermal=True, device=device)

    def _forward(self, flux, tau):
        prm = dict(self.prm, flux=flux, tau=float(tau[0]), tau_T=float(tau[1]))
        self.L.set_params(prm)
        self.L.init(self.ini["rho"], self.ini["ux"], self.ini["uy"], self.ini["T"])
        J = self.L.record(self.nsteps, self.ckpt, self.x_dev, *self.w)
        self.generation += 1
        return J

    def J(self, flux, tau):
        global _FN
        if _FN is None:
            _FN = _make_function()
        return _FN.apply(flux, tau, self)

    def close(self):
        self.L.close()

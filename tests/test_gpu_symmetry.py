"""Square symmetry of the HIP two-phase path itself, independent of the oracle:
on a square periodic grid a state transposed (velocity components exchanged)
must step into the transposed result, since every stencil, force and moment of
the model acts on its own axis with the same weight (the MRT rates under the
reading that puts omega_q2 on q_x and q_y, Sec. 2.3 and Sec. 3).  The two runs
of a pair sum in different orders, so they agree to FP64 rounding, not bit for
bit: u to the FP64 resolution of the gas velocity (u_tol: rounding of the
pressure populations divided by rho_g, as in the parity tests; about 8e-12
m/s here), phi to 1e-13 and p to 1e-12 of max |p| (the oracle's own transposed
runs: 3e-15 m/s, 2e-15 and 7e-15).  The bubble starts at rest in pressure with
small random velocities; a random pressure field in the gas drives a transient
near the lattice speed that amplifies rounding to 1e-9 of the velocity, in the
oracle as well.  The interface-normal guard is raised (1e-3 / dx) so that no
bulk node flips its normal between the two runs.  Checked with the single-step
kernel and with the two-step kernel on whole rows."""
import numpy as np
import pytest

from paper_2302_04120_amd import workloads as WL

from gpu_cases import print_case, u_tol

pytestmark = pytest.mark.gpu


def _transpose(a):
    return np.ascontiguousarray(np.swapaxes(a, -1, -2))


@pytest.mark.parametrize("fusion", [1, 2])
def test_transposed_state_steps_into_the_transposed_result(fusion):
    from paper_2302_04120_amd import lbm
    print_case(test="transpose-symmetry", fusion=fusion)
    n, steps = 64, 60
    prm, ini, _ = WL.bubble(n=n, radii=(14,), batch=1, seed=4)
    prm["normal_eps"] = 1e-3 / prm["dx"]
    g = WL.rng(11)
    ux0 = g.uniform(-1e-3, 1e-3, (1, n, n))
    uy0 = g.uniform(-1e-3, 1e-3, (1, n, n))
    p0 = ini["p"]
    phi0 = ini["phi"]

    def run(phi, p, ux, uy):
        L = lbm.Lattice("phase", n, n, batch=1, prec="fp64")
        L.set_step_fusion(fusion)
        L.set_params(prm)
        L.init(p, ux, uy, None, phi)
        L.step(steps)
        m = L.macros(("phi", "p", "ux", "uy"))
        L.close()
        return m

    a = run(phi0, p0, ux0, uy0)
    b = run(_transpose(phi0), _transpose(p0), _transpose(uy0), _transpose(ux0))
    du = max(np.abs(a["ux"] - _transpose(b["uy"])).max(),
             np.abs(a["uy"] - _transpose(b["ux"])).max())
    dphi = np.abs(a["phi"] - _transpose(b["phi"])).max()
    dp = np.abs(a["p"] - _transpose(b["p"])).max() / np.abs(a["p"]).max()
    tol = u_tol(prm, a, "fp64")
    print("transpose deviation: u %.2e m/s (bound %.2e), phi %.2e, p %.2e" % (du, tol, dphi, dp))
    assert du < tol and dphi < 1e-13 and dp < 1e-12

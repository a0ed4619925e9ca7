"""Pins of the oracle's 3D momentum model: D3Q19 with the dimensional MRT of
Sec. 3 carried to three dimensions (the extension the paper calls direct in
its conclusions) and its BGK counterpart, with Guo forcing and
halfway bounce-back walls.

What fixes the numbers here, independently of the oracle's own code:
  * the moment basis of d'Humieres et al. (2002), orthogonal with their
    published row norms, and their published equilibrium moments
    e = -11 rho + 19 rho u^2, eps = 3 rho - 11/2 rho u^2, q = -2/3 j, ...;
  * linear hydrodynamics of the lattice: shear waves decay at nu k^2, sound
    travels at c/sqrt(3) and is damped at (2/3 nu + zeta/2) k^2 with the bulk
    viscosity zeta = (2 c^2 / 9)(1/omega_e - dt/2) of the e-row rate;
  * the exact steady solution of force-driven flow between halfway
    bounce-back walls: the continuum parabola plus the wall slip
    F dx^2 (16 Lambda - 3) / (24 rho nu), Lambda = (1/s_even - 1/2)(1/s_odd - 1/2)
    (BGK: (tau/dt - 1/2)^2; the MRT rates of Sec. 3: 1/12);
  * the cubic symmetry of the lattice and the unit-free form of the scheme.
"""
import numpy as np
import pytest

import oracle as O

NORMS = [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]
ORDER = [0, 2, 4, 1, 3, 1, 3, 1, 3, 2, 4, 2, 4, 2, 2, 2, 3, 3, 3]


def _prm(dx=1e-4, nu=1e-6, tau_hat=0.8, rho=1000.0, **kw):
    dt = (tau_hat - 0.5) * dx * dx / (3 * nu)
    return dict(dx=dx, dt=dt, rho_ref=rho, nu=nu, **kw)


def _run(shape, prm, rho, ux, uy, uz, steps, **bc):
    nz, ny, nx = shape
    d = O.D3(nx, ny, nz, prm, **bc)
    d.init(rho, ux, uy, uz)
    d.step(steps)
    return d


def test_basis_is_dhumieres_orthogonal_set():
    """M M^T is diagonal with the published norms; the dimensional matrix is
    the lattice one with row k scaled by c^order(k) (Eq. M_matrix_dim's rule),
    and its inverse is exact."""
    M1, _ = O.d3_mdim(1.0)
    np.testing.assert_allclose(M1 @ M1.T, np.diag(NORMS), atol=1e-12)
    c = 7.25
    Mc, Mci = O.d3_mdim(c)
    np.testing.assert_allclose(Mc, np.diag(c ** np.array(ORDER, float)) @ M1, rtol=1e-15)
    np.testing.assert_allclose(Mci @ Mc, np.eye(19), atol=1e-12)
    # first row sums the populations, rows 3/5/7 are the momentum components
    assert np.all(M1[0] == 1)
    assert sorted(M1[3].tolist()) == [-1] * 5 + [0] * 9 + [1] * 5


def test_equilibrium_moments_are_the_published_ones():
    """The oracle's equilibrium populations (written by init) have the
    moments of d'Humieres et al. (2002) for D3Q19, in SI form: every
    moment of degree n carries c^n."""
    g = np.random.default_rng(1)
    prm = _prm()
    c = prm["dx"] / prm["dt"]
    sh = (2, 3, 4)
    rho = 1000 * (1 + 0.01 * g.standard_normal(sh))
    u = [0.05 * c * g.standard_normal(sh) for _ in range(3)]
    d = O.D3(4, 3, 2, prm)
    d.init(rho, *u)
    f = d.get_state().reshape(19, -1)
    M, _ = O.d3_mdim(c)
    m = M @ f
    r = rho.ravel()
    ux, uy, uz = (a.ravel() for a in u)
    uu = ux ** 2 + uy ** 2 + uz ** 2
    c2 = c * c
    expect = [r, r * (19 * uu - 11 * c2), r * (3 * c2 * c2 - 5.5 * c2 * uu),
              r * ux, -2 / 3 * c2 * r * ux, r * uy, -2 / 3 * c2 * r * uy, r * uz, -2 / 3 * c2 * r * uz,
              r * (2 * ux ** 2 - uy ** 2 - uz ** 2), -0.5 * c2 * r * (2 * ux ** 2 - uy ** 2 - uz ** 2),
              r * (uy ** 2 - uz ** 2), -0.5 * c2 * r * (uy ** 2 - uz ** 2),
              r * ux * uy, r * uy * uz, r * ux * uz, 0 * r, 0 * r, 0 * r]
    for k in range(19):
        scale = np.abs(r).max() * c ** ORDER[k]
        np.testing.assert_allclose(m[k], expect[k], rtol=0, atol=1e-13 * scale, err_msg="row %d" % k)


@pytest.mark.parametrize("mrt", [False, True])
def test_conservation_and_forcing_impulse(mrt):
    """Periodic box, random state, body force: the total mass is constant and
    the total momentum sum(c_i f_i) grows by F dt per node per step."""
    g = np.random.default_rng(2)
    prm = _prm(F=(30.0, -20.0, 10.0), omega_e=0.0)
    c = prm["dx"] / prm["dt"]
    sh = (5, 4, 6)
    rho = 1000 * (1 + 1e-3 * g.standard_normal(sh))
    u = [1e-3 * c * g.standard_normal(sh) for _ in range(3)]
    d = O.D3(6, 4, 5, prm, mrt=mrt)
    d.init(rho, *u)
    M, _ = O.d3_mdim(c)

    def totals():
        m = M @ d.get_state().reshape(19, -1)
        return m[0].sum(), np.array([m[3].sum(), m[5].sum(), m[7].sum()])

    m0, j0 = totals()
    d.step(25)
    m1, j1 = totals()
    assert m1 == pytest.approx(m0, rel=1e-14)
    np.testing.assert_allclose(j1 - j0, 25 * prm["dt"] * np.array(prm["F"]) * rho.size,
                               rtol=1e-9)


def _shear_decay(n, mrt, axis_k=2):
    prm = _prm()
    c = prm["dx"] / prm["dt"]
    sh = [1, 1, 1]
    sh[2 - axis_k] = n
    sh = tuple(sh)
    xk = (np.arange(n) + 0.5) * prm["dx"]
    k = 2 * np.pi / (n * prm["dx"])
    U = 1e-4 * c
    prof = U * np.sin(k * xk)
    # velocity across the wave vector: along x for a wave in z or y, along y for one in x
    ux = np.zeros(sh)
    uy = np.zeros(sh)
    (uy if axis_k == 0 else ux)[...] = prof.reshape(sh)
    steps = int(0.5 / (prm["nu"] * k * k) / prm["dt"])
    d = _run(sh, prm, np.full(sh, 1000.0), ux, uy, np.zeros(sh), steps, mrt=mrt)
    m = d.macros()
    v = (m["uy"] if axis_k == 0 else m["ux"]).ravel()
    amp = 2 * np.mean(v * np.sin(k * xk))
    rate = -np.log(amp / U) / (steps * prm["dt"])
    return rate / (prm["nu"] * k * k)


@pytest.mark.parametrize("mrt", [False, True])
def test_shear_wave_decays_at_nu_k2(mrt):
    """A sinusoidal shear wave decays at nu k^2 with a second-order lattice
    error: within 3 % at 16 nodes per wavelength and four times closer at 32."""
    r16 = _shear_decay(16, mrt)
    r32 = _shear_decay(32, mrt)
    assert abs(r16 - 1) < 3e-2
    assert 3.8 < (r16 - 1) / (r32 - 1) < 4.2
    # the same wave along x and along y (the lattice's cubic symmetry)
    assert _shear_decay(16, mrt, axis_k=0) == pytest.approx(r16, rel=1e-9)
    assert _shear_decay(16, mrt, axis_k=1) == pytest.approx(r16, rel=1e-9)


@pytest.mark.parametrize("we_hat", [1.0, 1.4, 0.7])
def test_sound_speed_and_bulk_viscosity_of_the_e_rate(we_hat):
    """A standing sound wave oscillates at k c/sqrt(3) and is damped at
    (2/3 nu + zeta/2) k^2 with zeta = (2 c^2/9)(1/omega_e - dt/2): the free
    e-row rate of the MRT sets the bulk viscosity."""
    from scipy.optimize import curve_fit
    n, nu = 32, 1e-6
    prm = _prm(nu=nu, omega_e=0.0)
    dt = prm["dt"]
    prm["omega_e"] = we_hat / dt
    c = prm["dx"] / dt
    k = 2 * np.pi / (n * prm["dx"])
    z = (np.arange(n) + 0.5) * prm["dx"]
    sh = (n, 1, 1)
    A = 1e-6
    d = O.D3(1, 1, n, prm)
    d.init((1000 * (1 + A * np.cos(k * z))).reshape(sh), np.zeros(sh), np.zeros(sh), np.zeros(sh))
    w = k * c / np.sqrt(3)
    nsteps = int(4 * 2 * np.pi / w / dt)
    amp = np.empty(nsteps)
    for s in range(nsteps):
        d.step(1)
        r = d.macros()["rho"].ravel()
        amp[s] = 2 * np.mean((r / 1000 - 1) * np.cos(k * z))
    t = (np.arange(nsteps) + 1) * dt
    f = lambda t, a, gam, om, ph: a * np.exp(-gam * t) * np.cos(om * t + ph)
    p, _ = curve_fit(f, t, amp, p0=(A, nu * k * k, w, 0.0))
    zeta = (2 * c * c / 9) * (1 / prm["omega_e"] - dt / 2)
    assert p[1] / k ** 2 == pytest.approx(2 / 3 * nu + zeta / 2, rel=3e-3)
    assert p[2] == pytest.approx(w, rel=2e-3)


@pytest.mark.parametrize("mrt,tau_hat,Lam", [
    (False, 1.0, 0.25), (False, 0.5 + np.sqrt(3) / 4, 3 / 16), (True, 0.8, 1 / 12), (True, 1.3, 1 / 12)])
@pytest.mark.parametrize("wall_axis,force_axis", [(2, 0), (1, 2), (0, 1)])
def test_poiseuille_between_halfway_walls_is_exact(mrt, tau_hat, Lam, wall_axis, force_axis):
    """Force-driven flow between two halfway bounce-back walls reaches the
    parabola F/(2 rho nu) s (H - s) plus the slip F dx^2 (16 Lambda - 3) /
    (24 rho nu) exactly (the magic Lambda = 3/16 puts the wall at the
    halfway point); the same for walls normal to x, y or z."""
    n, rho, nu, dx = 12, 1000.0, 1e-6, 1e-4
    F = [0.0, 0.0, 0.0]
    F[force_axis] = 0.1
    prm = _prm(dx=dx, nu=nu, tau_hat=tau_hat, rho=rho, F=tuple(F))
    sh = [2, 2, 2]
    sh[2 - wall_axis] = n
    sh = tuple(sh)
    bc = {ax: ("walls" if i == wall_axis else "periodic") for i, ax in enumerate(("bc_x", "bc_y", "bc_z"))}
    H = n * dx
    steps = int(7 * H * H / nu / prm["dt"])
    zero = np.zeros(sh)
    d = _run(sh, prm, np.full(sh, rho), zero, zero, zero, steps, mrt=mrt, **bc)
    m = d.macros()
    u = m[("ux", "uy", "uz")[force_axis]]
    u = np.moveaxis(u, 2 - wall_axis, 0).reshape(n, -1)
    s = (np.arange(n) + 0.5) * dx
    exact = 0.1 / (2 * rho * nu) * s * (H - s) + 0.1 * dx * dx * (16 * Lam - 3) / (24 * rho * nu)
    umax = exact.max()
    for col in u.T:
        np.testing.assert_allclose(col, exact, rtol=0, atol=1e-7 * umax)
    for other in set(range(3)) - {force_axis}:
        assert np.abs(m[("ux", "uy", "uz")[other]]).max() < 1e-9 * umax


def test_cubic_symmetry_of_the_collision():
    """Cycling the axes x -> y -> z of a random periodic state (velocities
    cycled with them) cycles the state after any number of steps: the MRT
    rates, the forcing and the streaming treat the three axes alike."""
    g = np.random.default_rng(4)
    prm = _prm(omega_e=0.0, F=(5.0, -3.0, 2.0))
    prm["omega_e"] = 1.3 / prm["dt"]
    prm["omega_eps"] = 0.9 / prm["dt"]
    c = prm["dx"] / prm["dt"]
    n = 5
    sh = (n, n, n)
    rho = 1000 * (1 + 1e-3 * g.standard_normal(sh))
    ux, uy, uz = (1e-2 * c * g.standard_normal(sh) for _ in range(3))
    a = _run(sh, prm, rho, ux, uy, uz, 8).macros()
    # new axes: x' = z, y' = x, z' = y.  arrays are [z][y][x]
    cyc = lambda f: np.transpose(f, (1, 0, 2)).transpose(0, 2, 1)  # [z][y][x] -> [y][x][z]
    Fc = (prm["F"][2], prm["F"][0], prm["F"][1])
    b = _run(sh, dict(prm, F=Fc), cyc(rho), cyc(uz), cyc(ux), cyc(uy), 8).macros()
    np.testing.assert_allclose(b["rho"], cyc(a["rho"]), rtol=1e-13)
    sc = np.abs(a["ux"]).max()
    np.testing.assert_allclose(b["ux"], cyc(a["uz"]), atol=1e-12 * sc)
    np.testing.assert_allclose(b["uy"], cyc(a["ux"]), atol=1e-12 * sc)
    np.testing.assert_allclose(b["uz"], cyc(a["uy"]), atol=1e-12 * sc)


@pytest.mark.parametrize("mrt", [False, True])
def test_si_run_equals_lattice_unit_run(mrt):
    """Sec. 3's claim in 3D: the SI scheme with (dx, dt) and the lattice-unit
    scheme (dx = dt = 1, nu dt/dx^2, F dt^2/dx) give the same density and the
    same velocity up to the factor c = dx/dt."""
    g = np.random.default_rng(6)
    prm = _prm(F=(2.0, 1.0, -3.0))
    prm["omega_e"] = 1.2 / prm["dt"]
    dx, dt = prm["dx"], prm["dt"]
    c = dx / dt
    lu = dict(dx=1.0, dt=1.0, rho_ref=prm["rho_ref"], nu=prm["nu"] * dt / dx ** 2,
              F=tuple(f * dt * dt / dx for f in prm["F"]), omega_e=prm["omega_e"] * dt)
    sh = (4, 5, 6)
    rho = 1000 * (1 + 1e-3 * g.standard_normal(sh))
    u = [1e-2 * c * g.standard_normal(sh) for _ in range(3)]
    bc = dict(bc_y="walls", bc_z="walls", mrt=mrt)
    a = _run(sh, prm, rho, *u, 15, **bc).macros()
    b = _run(sh, lu, rho, *(x / c for x in u), 15, **bc).macros()
    np.testing.assert_allclose(a["rho"], b["rho"], rtol=1e-13)
    for k in ("ux", "uy", "uz"):
        np.testing.assert_allclose(a[k], c * b[k], atol=1e-11 * c * np.abs(b[k]).max())


def _duct_series(n, dx, F, rho, nu, terms=200):
    """Fully developed flow in a square duct of side a = n dx (no-slip walls),
    the classical Fourier series: u = 4 F a^2 / (mu pi^3) sum over odd k of
    (-1)^((k-1)/2) k^-3 [1 - cosh(k pi z / a) / cosh(k pi / 2)] cos(k pi y / a)."""
    a = n * dx
    s = (np.arange(n) + 0.5) * dx - a / 2
    Z, Y = np.meshgrid(s, s, indexing="ij")
    u = np.zeros_like(Y)
    for k in range(1, 2 * terms, 2):
        u += ((-1) ** ((k - 1) // 2) * (1 - np.cosh(k * np.pi * Z / a) / np.cosh(k * np.pi / 2))
              * np.cos(k * np.pi * Y / a) / k ** 3)
    return 4 * F * a * a / (rho * nu * np.pi ** 3) * u


@pytest.mark.parametrize("mrt,tau_hat", [(False, 0.5 + np.sqrt(3) / 4), (False, 1.0), (True, 0.8)])
def test_square_duct_flow_converges_to_the_series(mrt, tau_hat):
    """Walls on y and z at once (edges where diagonal links bounce back on two
    sides): the steady duct flow converges at second order to the series
    solution; within 0.5 % of the peak at 16 nodes per side."""
    errs = []
    for n in (8, 16):
        rho, nu, dx, F = 1000.0, 1e-6, 1e-4, 0.1
        prm = _prm(dx=dx, nu=nu, tau_hat=tau_hat, rho=rho, F=(F, 0.0, 0.0))
        sh = (n, n, 1)
        zero = np.zeros(sh)
        d = _run(sh, prm, np.full(sh, rho), zero, zero, zero, int(3 * (n * dx) ** 2 / nu / prm["dt"]),
                 bc_y="walls", bc_z="walls", mrt=mrt)
        u = d.macros()["ux"][:, :, 0]
        ex = _duct_series(n, dx, F, rho, nu)
        errs.append(np.abs(u - ex).max() / ex.max())
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 3.0


@pytest.mark.parametrize("mrt", [True, False])
def test_each_moment_of_a_uniform_state_relaxes_at_its_rate(mrt):
    """A uniform state on a periodic box streams into itself, so a step is a
    bare collision (no force).  Perturbed along one non-conserved row k of
    the basis, f = f_eq + eps c^order_k M^-1 e_k, the conserved moments and
    so f_eq stay put, and the perturbation of row k shrinks by exactly
    1 - s_k per step with no other row excited (Eq. colisao_MRT is diagonal
    in the moment basis).  This holds every rate, including the eps, pi and m
    rows that no hydrodynamic pin reaches.  Expected rates (the reading of
    Sec. 3 in the d'Humieres basis): e and eps at omega_e dt and omega_eps
    dt, the five stresses at dt/tau, pi at 1, q and m at the s_q with
    (1/s_nu - 1/2)(1/s_q - 1/2) = 1/12 (the Lambda of the Poiseuille pin);
    BGK: every non-conserved row at dt/tau."""
    prm = _prm(tau_hat=0.8, omega_e=0.0, omega_eps=0.0)
    dt = prm["dt"]
    prm["omega_e"], prm["omega_eps"] = 1.3 / dt, 0.7 / dt
    c = prm["dx"] / dt
    s_nu = 1.0 / 0.8
    s_q = 1.0 / (0.5 + (1.0 / 12.0) / (1.0 / s_nu - 0.5))
    if mrt:
        s = [None, 1.3, 0.7, None, s_q, None, s_q, None, s_q, s_nu, 1.0, s_nu, 1.0, s_nu, s_nu,
             s_nu, s_q, s_q, s_q]
    else:
        s = [None if k in (0, 3, 5, 7) else s_nu for k in range(19)]
    M, Mi = O.d3_mdim(c)
    scale = np.array([c ** o for o in ORDER])
    o = O.D3(2, 2, 2, prm, mrt=mrt)
    o.init(np.full((2, 2, 2), 1000.2), np.full((2, 2, 2), 2e-3), np.full((2, 2, 2), -1e-3),
           np.full((2, 2, 2), 1.5e-3))
    f0 = o.get_state()
    m0 = np.einsum("ki,izyx->kzyx", M, f0) / scale[:, None, None, None]
    eps = 1e-3 * 1000.0
    for k in range(19):
        if s[k] is None:
            continue
        o.set_state(f0 + eps * scale[k] * Mi[:, k][:, None, None, None])
        for n in (1, 2):
            o.step(1)
            m = np.einsum("ki,izyx->kzyx", M, o.get_state()) / scale[:, None, None, None]
            dm = (m - m0) / eps
            want = np.zeros(19)
            want[k] = (1.0 - s[k]) ** n
            np.testing.assert_allclose(dm, np.broadcast_to(want[:, None, None, None], dm.shape),
                                       rtol=0, atol=1e-9, err_msg="row %d, step %d" % (k, n))

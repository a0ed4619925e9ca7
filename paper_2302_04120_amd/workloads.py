"""Seeded synthetic workloads shaped like the paper's cases (arXiv 2302.04120).

This module holds no lattice-Boltzmann arithmetic.  It only produces SI input
values (property presets and discretisation choices) and the initial
macroscopic fields, with numpy's PCG64 generator and a stated seed, so that
the HIP path and the CPU oracle receive identical inputs.  Every entry states
which case of the paper it is shaped after.

All arrays are float64 in [ny][nx] layout (x fastest); batched fields are
[batch][ny][nx].  Parameter dicts use SI units throughout.
"""
import math

import numpy as np

# --------------------------------------------------------------------------
# Property presets (values printed in the paper's property tables)
# --------------------------------------------------------------------------

#: water at 301 K and 1 atm (Sec. 4.2, property table of the heated channel)
WATER_301K = dict(rho=996.279, nu=8.382e-7, k=0.611, cp=4180.333, alpha=1.467e-7)

#: the four two-phase systems of the static bubble (Sec. 4.3 property table);
#: nu in m^2/s, zeta in Pa s, sigma in N/m
TWO_PHASE_SYSTEMS = {
    "air_water_25C": dict(rho_g=1.184, rho_l=997.048, nu_g=155.770e-7, nu_l=8.927e-7,
                          zeta_g=1.845e-5, zeta_l=89.006e-5, sigma=0.072),
    "sat_water_100C": dict(rho_g=0.598, rho_l=958.349, nu_g=204.493e-7, nu_l=2.938e-7,
                           zeta_g=1.223e-5, zeta_l=28.158e-5, sigma=0.059),
    "sat_water_80C": dict(rho_g=0.294, rho_l=971.766, nu_g=392.919e-7, nu_l=3.643e-7,
                          zeta_g=1.154e-5, zeta_l=35.404e-5, sigma=0.063),
    "sat_water_25C": dict(rho_g=0.023, rho_l=997.003, nu_g=4204.120e-7, nu_l=8.927e-7,
                          zeta_g=0.970e-5, zeta_l=89.004e-5, sigma=0.072),
}


#: interface-normal guard: n = 0 where |grad phi| <= NORMAL_EPS_NODES / dx.  The
#: paper zeroes n only where the gradient is exactly zero; a threshold well
#: above FP32 rounding of phi keeps both precisions on the same side of it.
NORMAL_EPS_NODES = 1e-6


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def node_centres(n, dx):
    """Halfway (link-wise) placement: node j sits at (j + 1/2) dx (Sec. 2.1)."""
    return (np.arange(n) + 0.5) * dx


def poiseuille_profile(y, H, u_m):
    """Developed channel velocity, Eq. velocity_prof."""
    eta = y / H
    return 6.0 * u_m * (eta - eta * eta)


def developed_temperature_profile(y, H, T_in, q_s, k):
    """Developed channel temperature under uniform flux, Eq. temp_prof; its
    constant 0.243 is 17/70 to the printed precision, which makes the
    mixing-cup mean equal to T_in."""
    eta = y / H
    return T_in + q_s * H / k * (-(eta ** 4) + 2 * eta ** 3 - eta + 17.0 / 70.0)


def tanh_profile(gamma, W):
    """Planar equilibrium order parameter, Eq. diffuse_interface."""
    return 0.5 + 0.5 * np.tanh(2.0 * gamma / W)


# --------------------------------------------------------------------------
# C1: 1D slab with uniform volumetric source (Sec. 4.1 machinery)
# --------------------------------------------------------------------------

def slab_1d(seed=0, n=101, L=0.1, alpha=1e-5, k=1.0, qvol=1e4, T_wall=300.0, dt=1e-2,
            noise=0.1):
    dx = L / (n - 1)  # wet nodes x_i = i dx spanning [0, L]
    rho_cp = k / alpha
    T0 = np.full(n, T_wall)
    T0[1:-1] += rng(seed).uniform(-noise, noise, n - 2)
    prm = dict(dx=dx, dt=dt, alpha=alpha, rho_cp=rho_cp, T0=T_wall, TL=T_wall, k=k, L=L,
               qvol=qvol)
    return prm, T0


# --------------------------------------------------------------------------
# C2 / C5: heated plane channel, D2Q9 flow + D2Q5 thermal (Sec. 4.2)
# --------------------------------------------------------------------------

def channel(nx=800, ny=40, dx=2.5e-5, nu=1e-6, Pr=7.0, Re=50.0, q_s=1e4, T_in=300.0,
            tau_ratio=0.64, oscillating=False, developed=True, seed=0):
    """Full channel of height H = ny dx between two heated halfway walls.

    Re is based on the hydraulic diameter 2H; dt follows from tau/dt for the
    viscosity; the inlet carries the developed velocity and (when
    ``developed``) the developed temperature profile; the flow field starts
    either developed everywhere or at rest (``developed=False``: u = 0
    inside, parabolic inlet).  ``seed`` is unused (the case is deterministic)
    and kept for a uniform signature.
    """
    H = ny * dx
    L = nx * dx
    rho = WATER_301K["rho"]
    rho_cp = rho * WATER_301K["cp"]
    alpha = nu / Pr
    k = alpha * rho_cp
    u_m = Re * nu / (2.0 * H)
    dt = (tau_ratio - 0.5) * dx * dx / (3.0 * nu)
    y = node_centres(ny, dx)
    u_in = poiseuille_profile(y, H, u_m)
    T_prof = developed_temperature_profile(y, H, T_in, q_s, k) if developed else np.full(ny, T_in)
    prm = dict(dx=dx, dt=dt, rho_ref=rho, nu=nu, omega_e=1.0 / dt, omega_eps=1.0 / dt,
               Fx=0.0, Fy=0.0, alpha=alpha, rho_cp=rho_cp, qvol=0.0, T_ref=T_in,
               flux=np.full(nx, q_s), flux_amp=0.5 if oscillating else 0.0,
               flux_omega=2.0 * math.pi * u_m / L if oscillating else 0.0,
               inlet_u=u_in, inlet_T=T_prof, flow_mrt=1, thermal_mrt=1,
               k=k, H=H, L=L, u_m=u_m, q_s=q_s, T_in=T_in)
    rho0 = np.full((ny, nx), rho)
    if developed:
        ux0 = np.repeat(u_in[:, None], nx, axis=1)
    else:
        ux0 = np.zeros((ny, nx))
    uy0 = np.zeros((ny, nx))
    T0 = np.repeat(T_prof[:, None], nx, axis=1)
    return prm, dict(rho=rho0, ux=ux0, uy=uy0, T=T0)


def adjoint_channel(nx=1600, ny=80, dx=1.25e-5, **kw):
    """C5: the C2 channel at half the spacing, flow starting from rest."""
    return channel(nx=nx, ny=ny, dx=dx, developed=False, **kw)


# --------------------------------------------------------------------------
# C3: stationary bubble (Sec. 4.3)
# --------------------------------------------------------------------------

def bubble(n=256, radii=(20, 30, 40, 50), seed=0, dx=5e-6, dt=1e-7, W_nodes=4.0, M=1e-5,
           rho_l=1000.0, rho_g=0.0231, nu_l=8.927e-7, nu_g=4.20412e-4, sigma=0.07,
           batch=None, ny=None):
    """Periodic n x ny cell (ny = n by default) with one gas bubble (phi = 0
    inside), centre jittered by U(-1/2, 1/2) nodes per axis; one replica per
    radius (cycled when ``batch`` exceeds the number of radii).  p = 0 and u = 0
    initially."""
    if batch is None:
        batch = len(radii)
    if ny is None:
        ny = n
    g = rng(seed)
    X, Y = np.meshgrid(node_centres(n, dx), node_centres(ny, dx), indexing="xy")
    W = W_nodes * dx
    phi = np.zeros((batch, ny, n))
    centres = []
    for b in range(batch):
        R = radii[b % len(radii)] * dx
        jx, jy = g.uniform(-0.5, 0.5, 2)
        xc, yc = (n / 2 + jx) * dx, (ny / 2 + jy) * dx
        r = np.sqrt((X - xc) ** 2 + (Y - yc) ** 2)
        phi[b] = tanh_profile(r - R, W)  # gas inside the bubble
        centres.append((xc, yc, R))
    prm = dict(dx=dx, dt=dt, rho_l=rho_l, rho_g=rho_g, nu_l=nu_l, nu_g=nu_g,
               zeta_l=nu_l * rho_l, zeta_g=nu_g * rho_g, visc_mode=0, sigma=sigma, W=W, M=M,
               Fx=0.0, Fy=0.0, z_mrt=1, qy_printed=0, normal_eps=NORMAL_EPS_NODES / dx)
    zeros = np.zeros_like(phi)
    return prm, dict(phi=phi, p=zeros.copy(), ux=zeros.copy(), uy=zeros.copy()), centres


def bubble_array(cells=32, n=256, seed=0, **kw):
    """The bubble cell tiled into one periodic (cells n) x (cells n) domain:
    cell (i, j) (row i, column j) holds replica i cells + j of bubble(n,
    batch=cells^2, seed) -- radii cycling over 20/30/40/50 nodes, centre
    jitter drawn per cell.  The roofline-sized single-domain form of the
    bubble case (32 x 32 cells: 8192^2 nodes).  Returns (prm, ini, centres)
    with ini fields [1][cells n][cells n]."""
    prm, ini, cen = bubble(n=n, batch=cells * cells, seed=seed, **kw)
    out = {}
    for k, v in ini.items():
        out[k] = np.ascontiguousarray(
            v.reshape(cells, cells, n, n).transpose(0, 2, 1, 3).reshape(1, cells * n, cells * n))
    return prm, out, cen


# --------------------------------------------------------------------------
# C4: layered two-phase Poiseuille flow (Sec. 4.4)
# --------------------------------------------------------------------------

def layered(nx=4, ny=512, seed=0, dx=1.25e-6, dt=1.25e-8, W_nodes=20.0, M=1e-5,
            rho_l=1000.0, rho_g=0.0231, nu_l=8.927e-7, nu_g=4.20412e-4, sigma=0.07,
            u_c=1e-4, batch=1):
    """Liquid below the interface at y = H/2 + U(-1/2, 1/2) dx, gas above;
    halfway walls at y = 0 and y = H; driving force u_c (zeta_l + zeta_g) / h^2
    with h = H/2 (so that u_c is the interface speed of the sharp solution).
    The interface width defaults to the paper's W = 25 um (20 dx here)."""
    g = rng(seed)
    H = ny * dx
    h = 0.5 * H
    zeta_l, zeta_g = nu_l * rho_l, nu_g * rho_g
    Fx = u_c * (zeta_l + zeta_g) / (h * h)
    W = W_nodes * dx
    y = node_centres(ny, dx)
    phi = np.zeros((batch, ny, nx))
    offsets = []
    for b in range(batch):
        yi = h + g.uniform(-0.5, 0.5) * dx
        phi[b] = tanh_profile(yi - y, W)[:, None]  # liquid (phi = 1) below
        offsets.append(yi)
    prm = dict(dx=dx, dt=dt, rho_l=rho_l, rho_g=rho_g, nu_l=nu_l, nu_g=nu_g, zeta_l=zeta_l,
               zeta_g=zeta_g, visc_mode=1, sigma=sigma, W=W, M=M, Fx=Fx, Fy=0.0, z_mrt=1,
               qy_printed=0, H=H, h=h, u_c=u_c, normal_eps=NORMAL_EPS_NODES / dx)
    zeros = np.zeros_like(phi)
    return prm, dict(phi=phi, p=zeros.copy(), ux=zeros.copy(), uy=zeros.copy()), offsets


# --------------------------------------------------------------------------
# Natural convection in a square enclosure (App. D)
# --------------------------------------------------------------------------

AIR_333K = dict(rho=1.059, cp=1008.045, k=0.029, alpha=2.702e-5, nu=1.90e-5, beta=3.004e-3)


def cavity(Ra=1e4, dx=2e-4, dt=2e-4, n=None, g=9.81):
    """Square air-filled cavity: left wall hot, right wall cold, top and
    bottom insulated, fluid at rest at the cold temperature initially.
    Ra = 1e4: L = 13 mm, T_h = 373.15 K, T_c = 293.85 K; Ra = 1e6: L = 60 mm,
    T_h = 373.85 K, T_c = 293.15 K; properties at T_ref = 333.50 K.  (App. D
    prints L = 0.60 m for Ra = 1e6, which with its properties and wall
    temperatures gives Ra = 1.0e9; 0.060 m gives 1.0e6.)  ``n``
    overrides the node count across (L = n dx) for smaller test cavities
    with the same temperatures and properties."""
    if Ra == 1e4:
        L, Th, Tc = 0.0130, 373.15, 293.85
    elif Ra == 1e6:
        L, Th, Tc = 0.060, 373.85, 293.15
    else:
        raise ValueError("Ra must be 1e4 or 1e6")
    if n is None:
        n = int(round(L / dx))
    L = n * dx
    a = AIR_333K
    T_ref = 333.50
    prm = dict(dx=dx, dt=dt, rho_ref=a["rho"], nu=a["nu"], omega_e=1.0 / dt, omega_eps=1.0 / dt,
               Fx=0.0, Fy=0.0, alpha=a["alpha"], rho_cp=a["rho"] * a["cp"], qvol=0.0,
               T_ref=T_ref, flux=np.zeros(n), flux_amp=0.0, flux_omega=0.0,
               inlet_u=np.zeros(n), inlet_T=np.full(n, T_ref), flow_mrt=0, thermal_mrt=1,
               T_wall=(Th, Tc), beta_T=a["beta"], gravity=(0.0, -g),
               L=L, Th=Th, Tc=Tc,
               Ra=g * a["beta"] * L ** 3 * (Th - Tc) / (a["nu"] * a["alpha"]))
    ini = dict(rho=np.full((n, n), a["rho"]), ux=np.zeros((n, n)), uy=np.zeros((n, n)),
               T=np.full((n, n), Tc))
    return prm, ini


# --------------------------------------------------------------------------
# The paper's own heated-channel cases (Sec. 4.2): lower half of the channel
# with a symmetry plane at mid-height
# --------------------------------------------------------------------------

WATER_301K_SEC42 = dict(rho=996.279, nu=8.382e-7, k=0.611, cp=4180.333, alpha=1.467e-7)


def paper_channel(case, H=0.5e-3, L=10e-3, T_in=300.0, q_s=4e4, dq=4e4, L_h=1e-3):
    """case 'developed_alternating': developed inlet (Eq. velocity_prof with
    u_m = 0.2 m/s, Eq. temp_prof for the mean flux), flux q_s + dq sign(sin(2 pi
    x / L_h)) (Eq. var_flux), dx = 5 um, dt = 2 us.  'developing_constant':
    uniform inlet u_m = 0.02 m/s and T_in, flux q_s, dx = 2.5 um, dt = 0.625 us.
    'developing_alternating': the same with the alternating flux.  Grid: the
    lower half (H/2) of the channel, L long; BGK flow, D2Q9 MRT thermal."""
    w = WATER_301K_SEC42
    if case == "developed_alternating":
        dx, dt, u_m, developed, alternating = 5e-6, 2e-6, 0.2, True, True
    elif case == "developing_constant":
        dx, dt, u_m, developed, alternating = 2.5e-6, 6.25e-7, 0.02, False, False
    elif case == "developing_alternating":
        dx, dt, u_m, developed, alternating = 2.5e-6, 6.25e-7, 0.02, False, True
    else:
        raise ValueError(case)
    nx, ny = int(round(L / dx)), int(round(0.5 * H / dx))
    y = node_centres(ny, dx)
    x = node_centres(nx, dx)
    rho_cp = w["rho"] * w["cp"]
    k = w["k"]
    flux = q_s + (dq * np.sign(np.sin(2 * math.pi * x / L_h)) if alternating else 0.0 * x)
    if developed:
        u_in = poiseuille_profile(y, H, u_m)
        T_prof = developed_temperature_profile(y, H, T_in, q_s, k)
    else:
        u_in = np.full(ny, u_m)
        T_prof = np.full(ny, T_in)
    prm = dict(dx=dx, dt=dt, rho_ref=w["rho"], nu=w["nu"], omega_e=1.0 / dt, omega_eps=1.0 / dt,
               Fx=0.0, Fy=0.0, alpha=w["alpha"], rho_cp=rho_cp, qvol=0.0, T_ref=T_in,
               flux=flux, flux_amp=0.0, flux_omega=0.0, inlet_u=u_in, inlet_T=T_prof,
               flow_mrt=0, thermal_mrt=1, k=k, H=H, L=L, u_m=u_m, q_s=q_s, T_in=T_in)
    ux0 = np.repeat(u_in[:, None], nx, axis=1) if developed else np.zeros((ny, nx))
    ini = dict(rho=np.full((ny, nx), w["rho"]), ux=ux0, uy=np.zeros((ny, nx)),
               T=np.repeat(T_prof[:, None], nx, axis=1))
    return prm, ini


def box3d(nx=64, ny=64, nz=64, batch=1, seed=0, dx=1e-4, tau_ratio=0.8, fluid=None,
          u_frac=0.02, rho_frac=1e-3, F=(0.0, 0.0, 0.0), period=None, mrt=True):
    """A 3D box of water at 301 K (the fluid of Sec. 4.2) for the D3Q19 model:
    dt from tau / dt = tau_ratio, a random velocity field of rms u_frac * c and a
    random density perturbation rho_frac * rho.  ``period`` = (px, py) makes the
    fields periodic in x and y with that period (a small cell tiled over the
    box).  Arrays are [batch][nz][ny][nx]."""
    fl = fluid or WATER_301K
    nu = fl["nu"]
    dt = (tau_ratio - 0.5) * dx * dx / (3.0 * nu)
    c = dx / dt
    prm = dict(dx=dx, dt=dt, rho_ref=fl["rho"], nu=nu, F=tuple(F), flow_mrt=int(mrt))
    g = rng(seed)
    px, py = period if period is not None else (nx, ny)
    shape = (batch, nz, py, px)
    rho = fl["rho"] * (1.0 + rho_frac * g.standard_normal(shape))
    u = [u_frac * c * g.standard_normal(shape) for _ in range(3)]
    reps = (1, 1, ny // py, nx // px)
    tile = lambda a: np.tile(a, reps)
    ini = dict(rho=tile(rho), ux=tile(u[0]), uy=tile(u[1]), uz=tile(u[2]))
    return prm, ini


def bubble3d(n=64, ny=None, nz=None, R_nodes=12.0, shape="sphere", axis=2, seed=0, dx=5e-6,
             dt=1e-7, W_nodes=4.0, M=1e-5, rho_l=1000.0, rho_g=0.0231, nu_l=8.927e-7,
             nu_g=4.20412e-4, sigma=0.07, batch=1, u_noise=0.0, p_laplace=False):
    """The C3 bubble (air/water-like properties of the stationary-bubble case,
    Sec. 4.3) in a periodic 3D box: a gas sphere, or a gas cylinder whose axis
    runs along ``axis`` (0 x, 1 y, 2 z), radius R_nodes, centre jittered by
    U(-1/2, 1/2) nodes per axis.  p = 0, or with ``p_laplace`` the Laplace
    jump (2 sigma / R for the sphere, sigma / R for the cylinder) weighted by
    the gas fraction 1 - phi: started from p = 0, a large sphere's start-up
    pressure wave focuses at its centre and can push phi below -rho_g / drho,
    where the linear density law gives rho <= 0.  ``u_noise`` adds a seeded
    random velocity of that many m/s (rms per component).  Arrays
    [batch][nz][ny][nx]."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    g = rng(seed)
    Z, Y, X = np.meshgrid(node_centres(nz, dx), node_centres(ny, dx), node_centres(n, dx),
                          indexing="ij")
    W = W_nodes * dx
    phi = np.zeros((batch, nz, ny, n))
    for b in range(batch):
        j = g.uniform(-0.5, 0.5, 3)
        c = ((n / 2 + j[0]) * dx, (ny / 2 + j[1]) * dx, (nz / 2 + j[2]) * dx)
        d = [(X - c[0]) ** 2, (Y - c[1]) ** 2, (Z - c[2]) ** 2]
        if shape == "cylinder":
            d[axis] = 0.0 * d[axis]
        r = np.sqrt(d[0] + d[1] + d[2])
        phi[b] = tanh_profile(r - R_nodes * dx, W)
    prm = dict(dx=dx, dt=dt, rho_l=rho_l, rho_g=rho_g, nu_l=nu_l, nu_g=nu_g,
               zeta_l=nu_l * rho_l, zeta_g=nu_g * rho_g, visc_mode=0, sigma=sigma, W=W, M=M,
               F=(0.0, 0.0, 0.0), z_mrt=1, normal_eps=NORMAL_EPS_NODES / dx)
    u = [u_noise * g.standard_normal(phi.shape) for _ in range(3)]
    jump = (1.0 if shape == "cylinder" else 2.0) * sigma / (R_nodes * dx)
    p = jump * (1.0 - phi) if p_laplace else np.zeros_like(phi)
    return prm, dict(phi=phi, p=p, ux=u[0], uy=u[1], uz=u[2])

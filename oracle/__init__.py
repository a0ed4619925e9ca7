"""FP64 CPU oracle of the dimensional lattice Boltzmann method -- TEST INFRASTRUCTURE.

Plain, slow, obviously-correct reference (arXiv 2302.04120) used only by the
tests, by the smoke check and by the CPU-baseline leg of the benchmark.  It
shares no code with the HIP library: the C source ``lbm_oracle.c`` is compiled
on its own with gcc and loaded here through ctypes; nothing here imports the
product package.

Parameters are plain dicts of SI values (the same keys the product binding
accepts); arrays are numpy float64 in [ny][nx] layout (x fastest).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = C.CDLL(_build.LIB)
        _declare(_lib)
    return _lib


def lib_omp():
    """The same oracle source built with its OpenMP row loops (the two-phase
    step on several threads; identical results)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_build.LIB_OMP):
            _build.build()
        _lib_omp = C.CDLL(_build.LIB_OMP)
        _declare(_lib_omp)
    return _lib_omp


_dp = C.POINTER(C.c_double)


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


class ChanParams(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("bc_x", C.c_int), ("bc_y", C.c_int),
                ("dx", C.c_double), ("dt", C.c_double),
                ("flow", C.c_int), ("flow_mrt", C.c_int),
                ("rho_ref", C.c_double), ("nu", C.c_double), ("omega_e", C.c_double),
                ("omega_eps", C.c_double), ("Fx", C.c_double), ("Fy", C.c_double),
                ("thermal", C.c_int), ("thermal_mrt", C.c_int),
                ("alpha", C.c_double), ("rho_cp", C.c_double), ("qdot", C.c_double),
                ("T_ref", C.c_double), ("flux_amp", C.c_double), ("flux_omega", C.c_double),
                ("Tw_x", C.c_double * 2), ("buoy", C.c_double * 2)]


class PhaseParams(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("bc_y", C.c_int),
                ("dx", C.c_double), ("dt", C.c_double),
                ("rho_l", C.c_double), ("rho_g", C.c_double), ("nu_l", C.c_double),
                ("nu_g", C.c_double), ("zeta_l", C.c_double), ("zeta_g", C.c_double),
                ("visc_mode", C.c_int), ("sigma", C.c_double), ("W", C.c_double),
                ("M", C.c_double), ("Fbx", C.c_double), ("Fby", C.c_double),
                ("z_mrt", C.c_int), ("qy_printed", C.c_int), ("normal_eps", C.c_double)]


class D3Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("bc_x", C.c_int), ("bc_y", C.c_int),
                ("bc_z", C.c_int), ("dx", C.c_double), ("dt", C.c_double), ("mrt", C.c_int),
                ("rho_ref", C.c_double), ("nu", C.c_double), ("omega_e", C.c_double),
                ("omega_eps", C.c_double), ("F", C.c_double * 3)]


class P3Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("bc_x", C.c_int),
                ("bc_y", C.c_int), ("bc_z", C.c_int), ("dx", C.c_double), ("dt", C.c_double),
                ("rho_l", C.c_double), ("rho_g", C.c_double), ("nu_l", C.c_double),
                ("nu_g", C.c_double), ("zeta_l", C.c_double), ("zeta_g", C.c_double),
                ("visc_mode", C.c_int), ("sigma", C.c_double), ("W", C.c_double),
                ("M", C.c_double), ("Fb", C.c_double * 3), ("z_mrt", C.c_int),
                ("normal_eps", C.c_double)]


_variants = {}


def _variant(path):
    if path not in _variants:
        L = C.CDLL(path)
        _declare(L)
        _variants[path] = L
    return _variants[path]


def _declare(L):
    L.orc_set_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_d1_run.restype = C.c_int
    L.orc_d1_run.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                             C.c_double, C.c_double, C.c_double, _dp, C.c_long, _dp]
    L.orc_mdim.argtypes = [C.c_double, _dp, _dp]
    L.orc_chan_create.restype = C.c_void_p
    L.orc_chan_create.argtypes = [C.POINTER(ChanParams), _dp, _dp, _dp]
    L.orc_chan_destroy.argtypes = [C.c_void_p]
    L.orc_chan_init.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.orc_chan_step.argtypes = [C.c_void_p, C.c_long]
    L.orc_chan_macros.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.orc_chan_time.restype = C.c_long
    L.orc_chan_time.argtypes = [C.c_void_p]
    L.orc_chan_get_state.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_chan_set_state.argtypes = [C.c_void_p, _dp, _dp, C.c_long]
    L.orc_chan_set_flux.argtypes = [C.c_void_p, _dp]
    L.orc_chan_set_tau.argtypes = [C.c_void_p, C.c_double, C.c_double]
    L.orc_chan_nusselt.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_chan_objective.restype = C.c_double
    L.orc_chan_objective.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
    L.orc_chan_adjoint.restype = C.c_int
    L.orc_chan_adjoint.argtypes = [C.c_void_p, C.c_long, C.c_int, C.c_int, C.c_double,
                                   C.c_double, _dp, _dp, _dp]
    L.orc_phase_create.restype = C.c_void_p
    L.orc_phase_create.argtypes = [C.POINTER(PhaseParams)]
    L.orc_phase_destroy.argtypes = [C.c_void_p]
    L.orc_phase_init.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.orc_phase_step.argtypes = [C.c_void_p, C.c_long]
    L.orc_phase_macros.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_phase_get_state.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_phase_gradients.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_phase_set_state.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_d3_mdim.argtypes = [C.c_double, _dp, _dp]
    L.orc_d3_create.restype = C.c_void_p
    L.orc_d3_create.argtypes = [C.POINTER(D3Params)]
    L.orc_d3_destroy.argtypes = [C.c_void_p]
    L.orc_d3_init.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.orc_d3_step.argtypes = [C.c_void_p, C.c_long]
    L.orc_d3_macros.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.orc_d3_get_state.argtypes = [C.c_void_p, _dp]
    L.orc_d3_set_state.argtypes = [C.c_void_p, _dp]
    L.orc_p3_create.restype = C.c_void_p
    L.orc_p3_create.argtypes = [C.POINTER(P3Params)]
    L.orc_p3_destroy.argtypes = [C.c_void_p]
    L.orc_p3_init.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp]
    L.orc_p3_step.argtypes = [C.c_void_p, C.c_long]
    L.orc_p3_macros.argtypes = [C.c_void_p] + [_dp] * 7
    L.orc_p3_gradients.argtypes = [C.c_void_p] + [_dp] * 4
    L.orc_p3_get_state.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_p3_set_state.argtypes = [C.c_void_p, _dp, _dp, _dp]


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = np.broadcast_to(a, shape).copy()
    return a


def d1_run(q, n, dx, dt, alpha, qdot, T0, TL, T_init, nsteps, u=0.0):
    """1D thermal BGK (D1Q2 or D1Q3) with wet-node Dirichlet ends; returns T [n]."""
    T_init = _f64(T_init, (n,))
    out = np.zeros(n)
    rc = lib().orc_d1_run(q, n, dx, dt, alpha, qdot, u, T0, TL, _ptr(T_init), int(nsteps),
                          _ptr(out))
    if rc != 0:
        raise ValueError("orc_d1_run failed: %d" % rc)
    return out


def mdim(c):
    """Dimensional D2Q9 matrix M_dim and its numerical inverse (9x9 each)."""
    M = np.zeros((9, 9))
    Mi = np.zeros((9, 9))
    lib().orc_mdim(c, _ptr(M), _ptr(Mi))
    return M, Mi


class Chan:
    """D2Q9 flow (BGK/MRT) + optional thermal field on an nx x ny grid.

    ``bc_x``: 'periodic', 'inlet_outlet' or 'walls_T' (no-slip walls held at
    prm['T_wall'] = (T at x-, T at x+), App. D); ``bc_y``: 'periodic',
    'walls' or 'wall_symmetry' (wall at y-, symmetry plane at y+: the lower
    half of a channel).  ``thermal``: False, True or 'd2q5' (D2Q5), 'd2q9'.  prm['beta_T'] (1/K) with prm['gravity'] (m/s^2) adds the
    Boussinesq force -rho_ref beta (T - T_ref) g of Eq. buoyancy_force.
    """

    def __init__(self, nx, ny, prm, bc_x="periodic", bc_y="periodic", flow=True,
                 thermal=False):
        self.nx, self.ny = nx, ny
        P = ChanParams()
        P.nx, P.ny = nx, ny
        P.bc_x = {"periodic": 0, "inlet_outlet": 1, "walls_T": 2}[bc_x]
        P.bc_y = {"periodic": 0, "walls": 1, "wall_symmetry": 2}[bc_y]
        P.dx, P.dt = prm["dx"], prm["dt"]
        P.flow = 1 if flow else 0
        P.flow_mrt = int(prm.get("flow_mrt", 1))
        P.rho_ref = prm.get("rho_ref", 1.0)
        P.nu = prm.get("nu", 1e-6)
        P.omega_e = prm.get("omega_e", 1.0 / prm["dt"])
        P.omega_eps = prm.get("omega_eps", 1.0 / prm["dt"])
        P.Fx, P.Fy = prm.get("Fx", 0.0), prm.get("Fy", 0.0)
        P.thermal = {False: 0, True: 1, "d2q5": 1, "d2q9": 2}[thermal]
        self.qT = 9 if P.thermal == 2 else 5
        P.thermal_mrt = int(prm.get("thermal_mrt", 1))
        P.alpha = prm.get("alpha", 1e-7)
        P.rho_cp = prm.get("rho_cp", 1.0)
        # heat source in K/s from the volumetric rate, qdot = qvol / rho_cp (Eq. forcing_term_g)
        P.qdot = prm.get("qvol", 0.0) / P.rho_cp
        P.T_ref = prm.get("T_ref", 0.0)
        P.flux_amp = prm.get("flux_amp", 0.0)
        P.flux_omega = prm.get("flux_omega", 0.0)
        tw = prm.get("T_wall", (P.T_ref, P.T_ref))
        P.Tw_x[0], P.Tw_x[1] = tw[0], tw[1]
        # Boussinesq force per kelvin, -rho_ref beta g (Eq. buoyancy_force)
        beta = prm.get("beta_T", 0.0)
        gx, gy = prm.get("gravity", (0.0, 0.0))
        P.buoy[0], P.buoy[1] = -P.rho_ref * beta * gx, -P.rho_ref * beta * gy
        self.P = P
        flux = _f64(prm.get("flux", 0.0), (nx,))
        inlet_u = _f64(prm.get("inlet_u", 0.0), (ny,))
        inlet_T = _f64(prm.get("inlet_T", P.T_ref), (ny,))
        self.h = lib().orc_chan_create(C.byref(P), _ptr(flux), _ptr(inlet_u), _ptr(inlet_T))
        if not self.h:
            raise ValueError("orc_chan_create failed")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_chan_destroy(self.h)
            self.h = None

    def init(self, rho, ux, uy, T=None):
        sh = (self.ny, self.nx)
        lib().orc_chan_init(self.h, _ptr(_f64(rho, sh)), _ptr(_f64(ux, sh)), _ptr(_f64(uy, sh)),
                            _ptr(_f64(T, sh)) if T is not None else None)

    def step(self, n):
        lib().orc_chan_step(self.h, int(n))

    @property
    def t(self):
        return lib().orc_chan_time(self.h)

    def macros(self):
        sh = (self.ny, self.nx)
        r, a, b, T = (np.zeros(sh) for _ in range(4))
        lib().orc_chan_macros(self.h, _ptr(r), _ptr(a), _ptr(b), _ptr(T))
        return {"rho": r, "ux": a, "uy": b, "T": T}

    def get_state(self):
        f = np.zeros((9, self.ny, self.nx))
        g = np.zeros((self.qT, self.ny, self.nx))
        lib().orc_chan_get_state(self.h, _ptr(f), _ptr(g))
        return f, g

    def set_state(self, f, g, t=0):
        lib().orc_chan_set_state(self.h, _ptr(_f64(f)), _ptr(_f64(g)), int(t))

    def set_flux(self, flux):
        lib().orc_chan_set_flux(self.h, _ptr(_f64(flux, (self.nx,))))

    def set_tau(self, nu, alpha):
        lib().orc_chan_set_tau(self.h, nu, alpha)

    def nusselt(self):
        Tb, Tw, Nu = (np.zeros(self.nx) for _ in range(3))
        lib().orc_chan_nusselt(self.h, _ptr(Tb), _ptr(Tw), _ptr(Nu))
        return Tb, Tw, Nu

    def objective(self, x_dev, w_tout=1.0, w_nu=1.0):
        return lib().orc_chan_objective(self.h, int(x_dev), w_tout, w_nu)

    def adjoint(self, nsteps, ckpt, x_dev, w_tout=1.0, w_nu=1.0):
        J = np.zeros(1)
        gq = np.zeros(self.nx)
        gt = np.zeros(2)
        rc = lib().orc_chan_adjoint(self.h, int(nsteps), int(ckpt), int(x_dev), w_tout, w_nu,
                                    _ptr(J), _ptr(gq), _ptr(gt))
        if rc != 0:
            raise ValueError("orc_chan_adjoint failed: %d" % rc)
        return J[0], gq, gt


class Phase:
    """Conservative Allen-Cahn h + pressure-evolution z on an nx x ny grid
    (x periodic; y periodic or halfway walls).  threads > 0 runs the step on
    that many threads (the OpenMP build of the same source); self.threads is
    the count in effect."""

    def __init__(self, nx, ny, prm, bc_y="periodic", threads=0, variant=None):
        self.nx, self.ny = nx, ny
        self._L = lib_omp() if threads > 0 else lib()
        if variant is not None:  # a copy built by build.build_variant (pin self-check)
            self._L = _variant(variant)
        self.threads = self._L.orc_set_threads(int(threads)) if threads > 0 else 1
        P = PhaseParams()
        P.nx, P.ny = nx, ny
        P.bc_y = {"periodic": 0, "walls": 1}[bc_y]
        P.dx, P.dt = prm["dx"], prm["dt"]
        for k in ("rho_l", "rho_g", "nu_l", "nu_g", "sigma", "W", "M"):
            setattr(P, k, prm[k])
        P.zeta_l = prm.get("zeta_l", prm["nu_l"] * prm["rho_l"])
        P.zeta_g = prm.get("zeta_g", prm["nu_g"] * prm["rho_g"])
        P.visc_mode = int(prm.get("visc_mode", 0))
        P.Fbx, P.Fby = prm.get("Fx", 0.0), prm.get("Fy", 0.0)
        P.z_mrt = int(prm.get("z_mrt", 1))
        P.qy_printed = int(prm.get("qy_printed", 0))
        P.normal_eps = prm.get("normal_eps", 1e-12 / prm["dx"])
        self.P = P
        self.h = self._L.orc_phase_create(C.byref(P))
        if not self.h:
            raise ValueError("orc_phase_create failed")

    def __del__(self):
        if getattr(self, "h", None):
            self._L.orc_phase_destroy(self.h)
            self.h = None

    def init(self, phi, p, ux, uy):
        sh = (self.ny, self.nx)
        self._L.orc_phase_init(self.h, _ptr(_f64(phi, sh)), _ptr(_f64(p, sh)), _ptr(_f64(ux, sh)),
                             _ptr(_f64(uy, sh)))

    def step(self, n):
        self._L.orc_phase_step(self.h, int(n))

    def macros(self):
        sh = (self.ny, self.nx)
        out = {k: np.zeros(sh) for k in ("phi", "rho", "p", "ux", "uy", "mu")}
        self._L.orc_phase_macros(self.h, *(_ptr(out[k]) for k in
                                         ("phi", "rho", "p", "ux", "uy", "mu")))
        return out

    def gradients(self):
        sh = (self.ny, self.nx)
        gx, gy, lap = np.zeros(sh), np.zeros(sh), np.zeros(sh)
        self._L.orc_phase_gradients(self.h, _ptr(gx), _ptr(gy), _ptr(lap))
        return gx, gy, lap

    def get_state(self):
        h = np.zeros((9, self.ny, self.nx))
        z = np.zeros((9, self.ny, self.nx))
        pu = np.zeros((2, self.ny, self.nx))
        self._L.orc_phase_get_state(self.h, _ptr(h), _ptr(z), _ptr(pu))
        return h, z, pu

    def set_state(self, h, z, pu):
        self._L.orc_phase_set_state(self.h, _ptr(_f64(h)), _ptr(_f64(z)), _ptr(_f64(pu)))


def d3_mdim(c):
    """The dimensional D3Q19 moment matrix and its inverse (Sec. 3 in 3D)."""
    M = np.zeros((19, 19))
    Mi = np.zeros((19, 19))
    lib().orc_d3_mdim(float(c), _ptr(M), _ptr(Mi))
    return M, Mi


class D3:
    """D3Q19 momentum (BGK or the dimensional MRT) on nx x ny x nz, arrays
    indexed [z][y][x]; each axis periodic or closed by halfway walls."""

    def __init__(self, nx, ny, nz, prm, bc_x="periodic", bc_y="periodic", bc_z="periodic",
                 mrt=True):
        self.shape = (nz, ny, nx)
        P = D3Params()
        P.nx, P.ny, P.nz = nx, ny, nz
        kinds = {"periodic": 0, "walls": 1}
        P.bc_x, P.bc_y, P.bc_z = kinds[bc_x], kinds[bc_y], kinds[bc_z]
        P.dx, P.dt, P.mrt = prm["dx"], prm["dt"], int(mrt)
        P.rho_ref, P.nu = prm["rho_ref"], prm["nu"]
        P.omega_e, P.omega_eps = prm.get("omega_e", 0.0), prm.get("omega_eps", 0.0)
        F = prm.get("F", (0.0, 0.0, 0.0))
        for i in range(3):
            P.F[i] = F[i]
        self.P = P
        self.h = lib().orc_d3_create(C.byref(P))
        if not self.h:
            raise ValueError("orc_d3_create failed")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_d3_destroy(self.h)
            self.h = None

    def init(self, rho, ux, uy, uz):
        sh = self.shape
        lib().orc_d3_init(self.h, *(_ptr(_f64(a, sh)) for a in (rho, ux, uy, uz)))

    def step(self, n):
        lib().orc_d3_step(self.h, int(n))

    def macros(self):
        out = {k: np.zeros(self.shape) for k in ("rho", "ux", "uy", "uz")}
        lib().orc_d3_macros(self.h, *(_ptr(out[k]) for k in ("rho", "ux", "uy", "uz")))
        return out

    def get_state(self):
        f = np.zeros((19,) + self.shape)
        lib().orc_d3_get_state(self.h, _ptr(f))
        return f

    def set_state(self, f):
        lib().orc_d3_set_state(self.h, _ptr(_f64(f, (19,) + self.shape)))


class Phase3:
    """3D two-phase model (Sec. 2.3 on D3Q19) on nx x ny x nz, arrays [z][y][x];
    each axis periodic or closed by halfway walls."""

    def __init__(self, nx, ny, nz, prm, bc_x="periodic", bc_y="periodic", bc_z="periodic"):
        self.shape = (nz, ny, nx)
        kinds = {"periodic": 0, "walls": 1}
        P = P3Params()
        P.nx, P.ny, P.nz = nx, ny, nz
        P.bc_x, P.bc_y, P.bc_z = kinds[bc_x], kinds[bc_y], kinds[bc_z]
        P.dx, P.dt = prm["dx"], prm["dt"]
        for k in ("rho_l", "rho_g", "nu_l", "nu_g", "sigma", "W", "M"):
            setattr(P, k, prm[k])
        P.zeta_l = prm.get("zeta_l", prm["nu_l"] * prm["rho_l"])
        P.zeta_g = prm.get("zeta_g", prm["nu_g"] * prm["rho_g"])
        P.visc_mode = int(prm.get("visc_mode", 0))
        F = prm.get("F", (prm.get("Fx", 0.0), prm.get("Fy", 0.0), prm.get("Fz", 0.0)))
        for a in range(3):
            P.Fb[a] = F[a]
        P.z_mrt = int(prm.get("z_mrt", 1))
        P.normal_eps = prm.get("normal_eps", 1e-12 / prm["dx"])
        self.P = P
        self.h = lib().orc_p3_create(C.byref(P))
        if not self.h:
            raise ValueError("orc_p3_create failed")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_p3_destroy(self.h)
            self.h = None

    def init(self, phi, p, ux, uy, uz):
        sh = self.shape
        lib().orc_p3_init(self.h, *(_ptr(_f64(a, sh)) for a in (phi, p, ux, uy, uz)))

    def step(self, n):
        lib().orc_p3_step(self.h, int(n))

    def macros(self):
        keys = ("phi", "rho", "p", "ux", "uy", "uz", "mu")
        out = {k: np.zeros(self.shape) for k in keys}
        lib().orc_p3_macros(self.h, *(_ptr(out[k]) for k in keys))
        return out

    def gradients(self):
        g = [np.zeros(self.shape) for _ in range(4)]
        lib().orc_p3_gradients(self.h, *(_ptr(a) for a in g))
        return g

    def get_state(self):
        h = np.zeros((19,) + self.shape)
        z = np.zeros((19,) + self.shape)
        pu = np.zeros((3,) + self.shape)
        lib().orc_p3_get_state(self.h, _ptr(h), _ptr(z), _ptr(pu))
        return h, z, pu

    def set_state(self, h, z, pu):
        sh = self.shape
        lib().orc_p3_set_state(self.h, _ptr(_f64(h, (19,) + sh)), _ptr(_f64(z, (19,) + sh)),
                               _ptr(_f64(pu, (3,) + sh)))


# --------------------------------------------------------------------------
# Diagnostics written from the paper's definitions (Sec. 4)
# --------------------------------------------------------------------------

def e2(ref, num):
    """Global relative L2 error in percent (Eq. error_norm_2)."""
    ref = np.asarray(ref, dtype=np.float64)
    num = np.asarray(num, dtype=np.float64)
    return 100.0 * np.sqrt(np.sum((ref - num) ** 2) / np.sum(ref ** 2))


def steady(chi_new, chi_old, tol):
    """Steady-state test of Eq. steady_state_cond: max change over 1000 steps."""
    return float(np.max(np.abs(np.asarray(chi_new) - np.asarray(chi_old)))) <= tol

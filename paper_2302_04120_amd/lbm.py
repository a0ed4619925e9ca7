"""Thin Python binding of liblbm.so (the C ABI of include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides the device buffer (one uint8 tensor of
``lbm_query_bytes`` bytes) and the HIP stream.  The binding never falls back
to anything else: if ``liblbm.so`` is missing or no GPU is visible it raises.

Parameter dicts use SI units and the keys of ``workloads``: dx, dt, rho_ref,
nu, omega_e, omega_eps, Fx, Fy, flow_mrt, thermal_mrt, T_ref, alpha, rho_cp,
qvol (W/m^3), flux, flux_amp, flux_omega, inlet_u, inlet_T, T0, TL, rho_l,
rho_g, nu_l, nu_g, zeta_l, zeta_g, visc_mode, sigma, W, M, z_mrt, qy_printed,
normal_eps, beta_T, gravity, T_wall, tau, tau_T; and for D3Q19 F = (Fx, Fy, Fz).
Every value is passed to the library as given (no unit conversion here).

Contexts are destroyed by ``Lattice.close()``, when the object is collected,
or at the latest by an exit hook that runs while the HIP runtime is still up.
"""
import atexit
import ctypes as C
import os
import warnings
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_E_ARG, LBM_E_TAU, LBM_E_DEVICE, LBM_E_STATE, LBM_E_NONFINITE, LBM_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
LBM_W_FP32_FORCING = 1  # informational bits: the call succeeded, see the warning text
LBM_W_MACH = 2
LBM_D1Q2, LBM_D1Q3, LBM_D2Q9_D2Q5, LBM_D2Q9_PHASE, LBM_D3Q19, LBM_D3Q19_PHASE = 1, 2, 3, 4, 5, 6
LBM_FP32_DEV, LBM_FP64, LBM_FP32_DEV_ARITH64 = 0, 1, 2
PRECISIONS = {"fp32": LBM_FP32_DEV, "fp64": LBM_FP64, "fp32_arith64": LBM_FP32_DEV_ARITH64}
BC_PERIODIC, BC_WALL, BC_VEL_INLET, BC_P_OUTLET, BC_DIRICHLET, BC_SYMMETRY = 0, 1, 2, 3, 4, 5
LBM_BGK, LBM_MRT = 0, 1
FLAG_FLOW, FLAG_THERMAL, FLAG_THERMAL_D2Q9 = 1, 2, 4
MACRO_BITS = {"rho": 1, "p": 2, "ux": 4, "uy": 8, "T": 16, "phi": 32, "mu": 64, "uz": 128}
REDUCE_BITS = {"mass": 1, "phase": 2, "energy": 4, "nonfinite": 8}

EXPORTS = ("lbm_query_bytes", "lbm_create", "lbm_destroy", "lbm_set_params_SI",
           "lbm_init_fields", "lbm_step", "lbm_macros", "lbm_reduce", "lbm_nusselt",
           "lbm_query_record_bytes", "lbm_record", "lbm_grad", "lbm_time",
           "lbm_save_state", "lbm_load_state", "lbm_last_error", "lbm_set_graph_steps",
           "lbm_set_step_fusion", "lbm_init_fields3d", "lbm_reduce_noalloc",
           "lbm_set_nonfinite_check", "lbm_first_nonfinite_step")


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("liblbm error %d: %s" % (status, msg))
        self.status = status


class Desc(C.Structure):
    _fields_ = [("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("batch", C.c_int),
                ("prec", C.c_int), ("bc", C.c_int * 4), ("flags", C.c_int),
                ("hip_stream", C.c_void_p), ("dev_buf", C.c_void_p), ("dev_buf_bytes", C.c_size_t),
                ("nz", C.c_int), ("bc_z", C.c_int * 2)]


_dp = C.POINTER(C.c_double)


class Objective(C.Structure):
    _fields_ = [("x_dev", C.c_int), ("w_tout", C.c_double), ("w_nu", C.c_double)]


class ParamsSI(C.Structure):
    _fields_ = [("dx", C.c_double), ("dt", C.c_double),
                ("flow_collision", C.c_int), ("rho_ref", C.c_double), ("nu", C.c_double),
                ("omega_e", C.c_double), ("omega_eps", C.c_double), ("Fb", C.c_double * 2),
                ("thermal_collision", C.c_int), ("T_ref", C.c_double), ("alpha", C.c_double),
                ("rho_cp", C.c_double), ("qvol", C.c_double), ("flux", _dp),
                ("flux_amp", C.c_double), ("flux_omega", C.c_double), ("inlet_u", _dp),
                ("inlet_T", _dp), ("T_wall", C.c_double * 2),
                ("rho_l", C.c_double), ("rho_g", C.c_double), ("nu_l", C.c_double),
                ("nu_g", C.c_double), ("zeta_l", C.c_double), ("zeta_g", C.c_double),
                ("visc_mode", C.c_int), ("sigma", C.c_double), ("W", C.c_double),
                ("mobility", C.c_double), ("z_collision", C.c_int), ("qy_printed", C.c_int),
                ("normal_eps", C.c_double), ("beta_T", C.c_double), ("gravity", C.c_double * 2),
                ("Fb_z", C.c_double), ("tau", C.c_double), ("tau_T", C.c_double)]


_lib = None


def lib():
    """Load liblbm.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm.so not built: run __graft_entry__.build() or "
                               "python paper_2302_04120_amd/csrc/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.lbm_query_bytes.argtypes = [C.POINTER(Desc), C.POINTER(C.c_size_t)]
        L.lbm_create.argtypes = [C.POINTER(Desc), C.POINTER(vp)]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        L.lbm_set_params_SI.argtypes = [vp, C.POINTER(ParamsSI)]
        L.lbm_init_fields.argtypes = [vp, _dp, _dp, _dp, _dp, _dp]
        L.lbm_init_fields3d.argtypes = [vp, _dp, _dp, _dp, _dp, _dp]
        L.lbm_step.argtypes = [vp, C.c_int]
        L.lbm_macros.argtypes = [vp, C.c_uint, _dp, C.c_int]
        L.lbm_reduce.argtypes = [vp, C.c_uint, _dp]
        L.lbm_reduce_noalloc.argtypes = [vp, C.c_uint, _dp]
        L.lbm_set_nonfinite_check.argtypes = [vp, C.c_int]
        L.lbm_first_nonfinite_step.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.lbm_nusselt.argtypes = [vp, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.lbm_time.argtypes = [vp]
        L.lbm_time.restype = C.c_longlong
        L.lbm_save_state.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.lbm_load_state.argtypes = [vp, vp, C.c_size_t]
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_query_record_bytes.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_size_t)]
        L.lbm_record.argtypes = [vp, C.c_int, C.c_int, C.POINTER(Objective), vp, C.c_size_t, _dp]
        L.lbm_grad.argtypes = [vp, C.c_double, _dp, _dp]
        L.lbm_set_graph_steps.argtypes = [vp, C.c_int]
        L.lbm_set_step_fusion.argtypes = [vp, C.c_int]
        for name in EXPORTS:
            if name not in ("lbm_destroy", "lbm_time", "lbm_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None:
        a = np.ascontiguousarray(np.broadcast_to(a, (n,)))
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def make_params(prm, nx=None, ny=None):
    """SI parameter dict -> ParamsSI (plus the arrays it points to, kept alive)."""
    P = ParamsSI()
    keep = []
    P.dx, P.dt = float(prm["dx"]), float(prm["dt"])
    P.flow_collision = LBM_MRT if int(prm.get("flow_mrt", 1)) else LBM_BGK
    P.rho_ref = float(prm.get("rho_ref", 1.0))
    P.nu = float(prm.get("nu", 1e-6))
    P.omega_e = float(prm.get("omega_e", 0.0))
    P.omega_eps = float(prm.get("omega_eps", 0.0))
    F = prm.get("F", (prm.get("Fx", 0.0), prm.get("Fy", 0.0), prm.get("Fz", 0.0)))
    P.Fb[0], P.Fb[1] = float(F[0]), float(F[1])
    P.Fb_z = float(F[2]) if len(F) > 2 else 0.0
    P.thermal_collision = LBM_MRT if int(prm.get("thermal_mrt", 1)) else LBM_BGK
    P.T_ref = float(prm.get("T_ref", 0.0))
    P.alpha = float(prm.get("alpha", 1e-7))
    P.rho_cp = float(prm.get("rho_cp", 1.0))
    P.qvol = float(prm.get("qvol", 0.0))
    for key in ("flux", "inlet_u", "inlet_T"):
        if prm.get(key) is not None:
            n = nx if key == "flux" else ny
            arr = _f64(prm[key], n)
            keep.append(arr)
            setattr(P, key, _ptr(arr))
    P.flux_amp = float(prm.get("flux_amp", 0.0))
    P.flux_omega = float(prm.get("flux_omega", 0.0))
    tw = prm.get("T_wall", (prm.get("T0", 0.0), prm.get("TL", 0.0)))
    P.T_wall[0], P.T_wall[1] = float(tw[0]), float(tw[1])
    P.beta_T = float(prm.get("beta_T", 0.0))
    gv = prm.get("gravity", (0.0, 0.0))
    P.gravity[0], P.gravity[1] = float(gv[0]), float(gv[1])
    for k in ("rho_l", "rho_g", "nu_l", "nu_g", "sigma", "W"):
        setattr(P, k, float(prm.get(k, 0.0)))
    P.zeta_l = float(prm.get("zeta_l", prm.get("nu_l", 0.0) * prm.get("rho_l", 0.0)))
    P.zeta_g = float(prm.get("zeta_g", prm.get("nu_g", 0.0) * prm.get("rho_g", 0.0)))
    P.visc_mode = int(prm.get("visc_mode", 0))
    P.mobility = float(prm.get("M", 0.0))
    P.z_collision = LBM_MRT if int(prm.get("z_mrt", 1)) else LBM_BGK
    P.qy_printed = int(prm.get("qy_printed", 0))
    P.normal_eps = float(prm.get("normal_eps", 0.0))
    P.tau = float(prm.get("tau", 0.0))
    P.tau_T = float(prm.get("tau_T", 0.0))
    return P, keep


# live contexts, destroyed at exit (before the interpreter tears torch down)
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for lat in list(_LIVE):
        lat.close()


class Lattice:
    """One lbm_ctx with its torch-owned device buffer and stream.

    lattice: 'd1q2' | 'd1q3' | 'channel' | 'phase' | 'd3q19' | 'phase3d'.  bc: 4 kinds
    (x-, x+, y-, y+), plus bc_z (z-, z+) and nz for the 3D lattices.
    prec: 'fp32' (FP32 deviation storage) | 'fp64' | 'fp32_arith64' (FP32 deviation
    storage, FP64 step arithmetic; two-phase D2Q9 only).
    """

    def __init__(self, lattice, nx, ny=1, batch=1, prec="fp32", bc=None, flow=True,
                 thermal=False, device="cuda:0", stream=None, nz=1, bc_z=(0, 0)):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a HIP device (torch.cuda.is_available() is False)")
        self.torch = torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        lat = {"d1q2": LBM_D1Q2, "d1q3": LBM_D1Q3, "channel": LBM_D2Q9_D2Q5,
               "phase": LBM_D2Q9_PHASE, "d3q19": LBM_D3Q19, "phase3d": LBM_D3Q19_PHASE}[lattice]
        if bc is None:
            bc = {"d1q2": (4, 4, 0, 0), "d1q3": (4, 4, 0, 0)}.get(lattice, (0, 0, 0, 0))
        d = Desc()
        d.lattice, d.nx, d.ny, d.batch = lat, nx, ny, batch
        if prec not in PRECISIONS:
            raise ValueError("prec must be one of %s" % sorted(PRECISIONS))
        d.prec = PRECISIONS[prec]
        for i in range(4):
            d.bc[i] = bc[i]
        three_d = lat in (LBM_D3Q19, LBM_D3Q19_PHASE)
        if three_d:
            d.nz = nz
            d.bc_z[0], d.bc_z[1] = bc_z
        # thermal: False, True / 'd2q5' (D2Q5), or 'd2q9' (D2Q9 thermal set)
        d.flags = ((FLAG_FLOW if flow and not three_d else 0) |
                   (FLAG_THERMAL if thermal else 0) | (FLAG_THERMAL_D2Q9 if thermal == "d2q9" else 0))
        d.hip_stream = C.c_void_p(self.stream.cuda_stream)
        nbytes = C.c_size_t()
        self._check(lib().lbm_query_bytes(C.byref(d), C.byref(nbytes)), None)
        self.buf = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        d.dev_buf = C.c_void_p(self.buf.data_ptr())
        d.dev_buf_bytes = nbytes.value
        self.desc = d
        h = C.c_void_p()
        self._check(lib().lbm_create(C.byref(d), C.byref(h)), None)
        self.ctx = h
        self._lib = lib()
        self.lattice, self.nx, self.ny, self.batch, self.prec = lattice, nx, ny, batch, prec
        self.nz = nz if three_d else 1
        self.bytes = int(nbytes.value)
        _LIVE.add(self)

    def _check(self, st, ctx="self"):
        """Raise LbmError on an error status; an informational one (a bit set
        of LBM_W_*, the call succeeded) is raised as a RuntimeWarning."""
        if st != LBM_OK:
            c = self.ctx if ctx == "self" else None
            msg = lib().lbm_last_error(c).decode() if c else "(no context)"
            if st > 0:
                warnings.warn("liblbm: " + msg, RuntimeWarning, stacklevel=3)
                return st
            raise LbmError(st, msg)
        return st

    def close(self):
        """Wait for the context's stream, destroy the context (its captured
        graphs and capture stream) and release the device buffers.  Idempotent."""
        L = getattr(self, "_lib", None)
        if getattr(self, "ctx", None) and L is not None:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            L.lbm_destroy(self.ctx)
            self.ctx = None
        self.buf = None
        self._work = None

    def __del__(self):
        # the library handle is held on the instance: at interpreter shutdown
        # the module globals may already be gone
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    @property
    def shape(self):
        if self.lattice in ("d3q19", "phase3d"):
            return (self.batch, self.nz, self.ny, self.nx)
        return (self.batch, self.ny, self.nx)

    def set_params(self, prm):
        """Returns the library status (LBM_OK, or a bit set of LBM_W_FP32_FORCING
        and LBM_W_MACH, also raised as a RuntimeWarning); errors raise LbmError."""
        P, keep = make_params(prm, self.nx, self.ny)
        st = lib().lbm_set_params_SI(self.ctx, C.byref(P))
        del keep
        return self._check(st)

    def init(self, rho_or_p=None, ux=None, uy=None, T=None, phi=None):
        n = self.batch * self.ny * self.nx
        arrs = [None if a is None else _f64(np.broadcast_to(np.asarray(a, dtype=np.float64),
                                                            self.shape).reshape(-1))
                for a in (rho_or_p, ux, uy, T, phi)]
        for a in arrs:
            assert a is None or a.size == n
        return self._check(lib().lbm_init_fields(self.ctx, *(_ptr(a) for a in arrs)))

    def init3d(self, rho_or_p=None, ux=None, uy=None, uz=None, phi=None):
        """3D lattices: equilibria of rho (D3Q19) or p and phi (phase3d) and u;
        arrays broadcast to [batch][nz][ny][nx]."""
        arrs = [None if a is None else _f64(np.broadcast_to(np.asarray(a, dtype=np.float64),
                                                            self.shape).reshape(-1))
                for a in (rho_or_p, ux, uy, uz, phi)]
        return self._check(lib().lbm_init_fields3d(self.ctx, *(_ptr(a) for a in arrs)))

    def step(self, n=1):
        self._check(lib().lbm_step(self.ctx, int(n)))

    def set_graph_steps(self, steps):
        """Steps per captured HIP graph replayed by ``step`` (0 disables)."""
        self._check(lib().lbm_set_graph_steps(self.ctx, int(steps)))

    def set_nonfinite_check(self, every):
        """Check the state for NaN/Inf every `every` steps inside step() (0: off)."""
        self._check(lib().lbm_set_nonfinite_check(self.ctx, int(every)))

    def first_nonfinite_step(self):
        """Step count at which the in-step check first saw a non-finite state, or -1."""
        s = C.c_longlong()
        st = lib().lbm_first_nonfinite_step(self.ctx, C.byref(s))
        if st not in (LBM_OK, LBM_E_NONFINITE):
            self._check(st)
        return int(s.value)

    def set_step_fusion(self, mode):
        """Two-phase kernel choice: 0 automatic, 1 single-step, 2 two-step,
        3 many steps per cooperative launch (grids of at most 16 tiles)."""
        self._check(lib().lbm_set_step_fusion(self.ctx, int(mode)))

    @property
    def t(self):
        return int(lib().lbm_time(self.ctx))

    def macros(self, fields=None):
        if fields is None:
            fields = {"channel": ("rho", "ux", "uy") + (("T",) if self.desc.flags & FLAG_THERMAL else ()),
                      "phase": ("rho", "p", "ux", "uy", "phi", "mu"),
                      "d3q19": ("rho", "ux", "uy", "uz"),
                      "phase3d": ("rho", "p", "ux", "uy", "uz", "phi", "mu")}.get(self.lattice, ("T",))
        mask = 0
        for f in fields:
            mask |= MACRO_BITS[f]
        order = [f for f in MACRO_BITS if mask & MACRO_BITS[f]]
        out = np.zeros((len(order),) + self.shape)
        self._check(lib().lbm_macros(self.ctx, mask, _ptr(out), 0))
        return {f: out[i] for i, f in enumerate(order)}

    def macros_device(self, fields):
        """Same as macros() but into a float64 torch tensor on the device (async)."""
        mask = 0
        for f in fields:
            mask |= MACRO_BITS[f]
        order = [f for f in MACRO_BITS if mask & MACRO_BITS[f]]
        out = self.torch.empty((len(order),) + self.shape, dtype=self.torch.float64,
                               device=self.device)
        self._check(lib().lbm_macros(self.ctx, mask, C.cast(out.data_ptr(), _dp), 1))
        return {f: out[i] for i, f in enumerate(order)}

    def reduce(self, fields=("mass", "phase", "energy", "nonfinite"), check=True):
        mask = 0
        for f in fields:
            mask |= REDUCE_BITS[f]
        order = [f for f in REDUCE_BITS if mask & REDUCE_BITS[f]]
        out = np.zeros((len(order), self.batch))
        st = lib().lbm_reduce(self.ctx, mask, _ptr(out))
        if st != LBM_E_NONFINITE or check:
            self._check(st)
        return {f: out[i] for i, f in enumerate(order)}

    def reduce_noalloc(self, fields=("mass", "phase", "energy", "nonfinite"), check=True):
        """reduce() through lbm_reduce_noalloc (static scratch, no allocation)."""
        mask = 0
        for f in fields:
            mask |= REDUCE_BITS[f]
        order = [f for f in REDUCE_BITS if mask & REDUCE_BITS[f]]
        out = np.zeros((len(order), self.batch))
        st = lib().lbm_reduce_noalloc(self.ctx, mask, _ptr(out))
        if st != LBM_E_NONFINITE or check:
            self._check(st)
        return {f: out[i] for i, f in enumerate(order)}

    def nusselt(self, x_dev):
        Tb, Tw, Nu = np.zeros(self.nx), np.zeros(self.nx), np.zeros(self.nx)
        nm, to = C.c_double(), C.c_double()
        self._check(lib().lbm_nusselt(self.ctx, int(x_dev), _ptr(Tb), _ptr(Tw), _ptr(Nu),
                                      C.byref(nm), C.byref(to)))
        return Tb, Tw, Nu, nm.value, to.value

    def record(self, nsteps, ckpt_every, x_dev, w_tout=1.0, w_nu=1.0):
        """Run nsteps keeping checkpoints for the adjoint; returns J."""
        nbytes = C.c_size_t()
        self._check(lib().lbm_query_record_bytes(self.ctx, int(nsteps), int(ckpt_every),
                                                 C.byref(nbytes)))
        if getattr(self, "_work", None) is None or self._work.numel() < nbytes.value:
            self._work = None
            self._work = self.torch.empty(int(nbytes.value), dtype=self.torch.uint8,
                                          device=self.device)
        obj = Objective(int(x_dev), float(w_tout), float(w_nu))
        J = C.c_double()
        self._check(lib().lbm_record(self.ctx, int(nsteps), int(ckpt_every), C.byref(obj),
                                     C.c_void_p(self._work.data_ptr()), self._work.numel(),
                                     C.byref(J)))
        return J.value

    def grad(self, dL_dJ=1.0):
        """Discrete adjoint of the last record(): (dJ/dflux[nx], dJ/dtau[2])."""
        gq = np.zeros(self.nx)
        gt = np.zeros(2)
        self._check(lib().lbm_grad(self.ctx, float(dL_dJ), _ptr(gq), _ptr(gt)))
        return gq, gt

    def save_state(self):
        n = C.c_size_t()
        self._check(lib().lbm_save_state(self.ctx, None, C.byref(n)))
        blob = C.create_string_buffer(n.value)
        self._check(lib().lbm_save_state(self.ctx, blob, C.byref(n)))
        return bytes(blob.raw[:n.value])

    def load_state(self, blob):
        self._check(lib().lbm_load_state(self.ctx, C.c_char_p(blob), len(blob)))

/*
 * lbm.h -- C ABI of the MI355X (gfx950) dimensional lattice Boltzmann library.
 *
 * The library advances the dimensional LBM of arXiv 2302.04120 -- the lattice
 * Boltzmann equation solved directly in SI units with dx, dt and c = dx/dt in
 * metres and seconds and every property physical (Sec. 3) -- with hand-written
 * HIP kernels.  Models (Sec. 2):
 *   LBM_D2Q9_D2Q5  : D2Q9 momentum (BGK or dimensional MRT, Guo forcing) plus
 *                    an optional D2Q5 temperature field with heat source
 *                    (Sec. 2.1, 2.2); halfway walls, velocity inlet, pressure
 *                    outlet, flux walls (Eq. BB_vel, anti_BB_vel, anti_BB_T,
 *                    BB_T and the first-order outlet extrapolation).
 *   LBM_D2Q9_PHASE : conservative Allen-Cahn order parameter h_i and pressure-
 *                    evolution populations z_i (Sec. 2.3), MRT for z_i in the
 *                    dimensional form of Sec. 3, BGK for h_i.
 *   LBM_D1Q2/D1Q3  : 1D thermal BGK with source and wet-node Dirichlet ends
 *                    (Sec. 2.2, App. B).
 *   LBM_D3Q19      : 3D momentum, BGK or the dimensional MRT of Sec. 3 carried
 *                    to three dimensions (moment basis of d'Humieres et al.
 *                    2002, row k scaled by c^order(k)), Guo forcing; each axis
 *                    periodic or closed by halfway walls (Eq. BB_vel, u_w = 0).
 *   LBM_D3Q19_PHASE: the two-phase model of Sec. 2.3 in 3D: h_i and z_i on
 *                    D3Q19, z_i with the dimensional MRT (rates as in 2D, row by
 *                    row: 1/dt on rho, e, eps, j, pi; omega_q2 on q and m; 1/tau
 *                    on the stresses), the isotropic D3Q19 stencils; each axis
 *                    periodic or walls.
 *
 * Conventions
 *   - Every host number is an SI double.  No lattice units cross this ABI.
 *   - Host arrays are float64, layout [batch][ny][nx] with x fastest
 *     ([batch][nz][ny][nx] for LBM_D3Q19), and are copied before the call
 *     returns; the caller keeps ownership.
 *   - Device memory is owned by the caller: lbm_query_bytes gives the size of
 *     the one device buffer (desc.dev_buf) the library works in.  The library
 *     never allocates device memory itself.  The buffer and the HIP stream
 *     (desc.hip_stream) must stay valid until lbm_destroy.
 *   - All device work is enqueued on desc.hip_stream.  Calls that return host
 *     data synchronise that stream; lbm_step only enqueues (except in step
 *     fusion mode 3, see lbm_set_step_fusion).
 *   - Every call returns an lbm_status; on error the context is unchanged
 *     (except that a failed many-steps launch drops the state) and
 *     lbm_last_error() describes the cause.  Argument checks happen before
 *     any device work.  A context is used by one host thread at a time.
 *   - Precision LBM_FP32_DEV stores populations in FP32 as deviations from
 *     w_i * X_ref (X_ref = rho_ref for momentum, T_ref for temperature, 0 for
 *     z_i and h_i) and collides in FP32; the rest population h_0 is kept as an
 *     FP32 hi/lo pair that carries the node's exact order-parameter balance.
 *     LBM_FP64 stores and collides in FP64.  LBM_FP32_DEV_ARITH64
 *     (LBM_D2Q9_PHASE only) keeps the FP32 storage but evaluates every step in
 *     FP64: in FP32 arithmetic the per-step force increment of a slow liquid
 *     layer at small dt falls below the resolution of the moments it is added
 *     to, and runs of 1e7 steps and more drift (the layered channel at the
 *     paper's finest grid: 9-12 % against FP64's 1.2 %; in this mode it
 *     matches FP64); the two-step kernel is not available in this mode.
 *     Reductions are FP64 in all modes.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#if defined(__GNUC__) || defined(__clang__)
#define LBM_API __attribute__((visibility("default")))
#else
#define LBM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_E_ARG = -1,         /* invalid argument, size or combination             */
    LBM_E_TAU = -2,         /* a relaxation time is not above dt/2 (Sec. 4 text on stability) */
    LBM_E_DEVICE = -3,      /* a HIP call failed                                  */
    LBM_E_STATE = -4,       /* wrong call order or malformed state blob           */
    LBM_E_NONFINITE = -5,   /* a NaN/Inf was found in the populations             */
    LBM_E_UNSUPPORTED = -6, /* combination not implemented                        */
    /* informational (> 0, a bit set of the values below): the call succeeded;
       lbm_last_error says why it is reported */
    LBM_W_FP32_FORCING = 1, /* lbm_set_params_SI, LBM_D2Q9_PHASE in LBM_FP32_DEV with a body
                               force: the slowest viscous mode (wall distance, or the period)
                               relaxes by nu dt k^2 < 2^-23 per step, so FP32 arithmetic rounds
                               the per-step force increments of long runs away; the parameters
                               are set, and LBM_FP32_DEV_ARITH64 avoids the drift          */
    LBM_W_MACH = 2          /* lbm_set_params_SI (the inlet profile of a flow channel with a
                               velocity inlet) or lbm_init_fields / lbm_init_fields3d (the
                               initial velocity): some |u| dt / dx exceeds 0.3, i.e. the Mach
                               number |u| / c_s exceeds 0.52, where the equilibria of
                               Eq. feq_geral, second order in u / c_s, are neither accurate
                               nor reliably stable (also set for a NaN speed)              */
} lbm_status;

enum { LBM_D1Q2 = 1, LBM_D1Q3 = 2, LBM_D2Q9_D2Q5 = 3, LBM_D2Q9_PHASE = 4, LBM_D3Q19 = 5,
       LBM_D3Q19_PHASE = 6 };
enum { LBM_FP32_DEV = 0, LBM_FP64 = 1, LBM_FP32_DEV_ARITH64 = 2 };
/* boundary kinds per side, order x-, x+, y-, y+ */
enum {
    LBM_BC_PERIODIC = 0,   /* Sec. 2.1, last paragraph                                */
    LBM_BC_WALL = 1,       /* halfway bounce-back (Eq. BB_vel, u_w = 0); thermal flux Eq. BB_T;
                              D3Q19 and D3Q19_PHASE: on any axis, both sides of it        */
    LBM_BC_VEL_INLET = 2,  /* x- only: Eq. BB_vel with the inlet profile; thermal Eq. anti_BB_T */
    LBM_BC_P_OUTLET = 3,   /* x+ only: Eq. anti_BB_vel; thermal first-order extrapolation */
    LBM_BC_DIRICHLET = 4,  /* 1D ends: wet-node fixed temperature (Eq. BCs_1D_advection_diffusion);
                              D2Q9_D2Q5 x sides (both): no-slip halfway wall (Eq. BB_vel)
                              held at T_wall by Eq. anti_BB_T (App. D)                    */
    LBM_BC_SYMMETRY = 5    /* D2Q9_D2Q5 y+ only, with LBM_BC_WALL at y-: symmetry plane of
                              Eq. simetria (the lower half of a channel)                   */
};
enum { LBM_BGK = 0, LBM_MRT = 1 };
/* desc.flags for LBM_D2Q9_D2Q5 */
enum { LBM_FLAG_FLOW = 1, LBM_FLAG_THERMAL = 2, LBM_FLAG_THERMAL_D2Q9 = 4 };

typedef struct {
    int lattice;            /* LBM_D1Q2 | LBM_D1Q3 | LBM_D2Q9_D2Q5 | LBM_D2Q9_PHASE | LBM_D3Q19
                               | LBM_D3Q19_PHASE                                            */
    int nx, ny, batch;      /* grid per replica (1D: ny = 1) and number of replicas         */
    int prec;               /* LBM_FP32_DEV | LBM_FP64 | LBM_FP32_DEV_ARITH64 (D2Q9_PHASE
                               only); 1D: LBM_FP64 only                                    */
    int bc[4];              /* x-, x+, y-, y+ ; see the enum above                           */
    int flags;              /* LBM_D2Q9_D2Q5: LBM_FLAG_FLOW | LBM_FLAG_THERMAL, plus
                               LBM_FLAG_THERMAL_D2Q9 for the D2Q9 thermal set (Sec. 3)     */
    void* hip_stream;       /* hipStream_t the library enqueues on (NULL = default stream)  */
    void* dev_buf;          /* caller-owned device memory of at least lbm_query_bytes()     */
    size_t dev_buf_bytes;
    int nz;                 /* 3D lattices: nodes in z; other lattices: 0 or 1               */
    int bc_z[2];            /* 3D lattices: z-, z+ (PERIODIC or WALL, both alike); else 0    */
} lbm_desc;

typedef struct {
    double dx, dt;          /* m, s */
    /* momentum (Sec. 2.1, Sec. 3) */
    int flow_collision;     /* LBM_BGK | LBM_MRT                                            */
    double rho_ref;         /* kg/m^3: reference density; also rho_w of inlet/outlet rules */
    double nu;              /* m^2/s  -> tau = nu / c_s^2 + dt/2 (Eq. eq_kinematic_viscosity) */
    double omega_e, omega_eps; /* 1/s, free MRT rates of e and eps (0 -> 1/dt)              */
    double Fb[2];           /* N/m^3 body force                                             */
    /* temperature (Sec. 2.2) */
    int thermal_collision;  /* LBM_BGK | LBM_MRT: j at 1/tau_T, the rest at 1/dt (D2Q5 two-rate;
                               D2Q9 Lambda_T,dim of Sec. 3)                                 */
    double T_ref;           /* K: deviation reference and datum of the advective equilibrium */
    double alpha;           /* m^2/s  -> tau_T = alpha / c_s^2 + dt/2                       */
    double rho_cp;          /* J/(m^3 K)                                                    */
    double qvol;            /* W/m^3 volumetric source; qdot = qvol / rho_cp (Eq. forcing_term_g) */
    const double* flux;     /* [nx] W/m^2 wall heat flux into the fluid, both walls (NULL = 0) */
    double flux_amp, flux_omega; /* q''(x,t) = flux[x] (1 + amp sin(omega t)), t = step * dt  */
    const double* inlet_u;  /* [ny] m/s inlet velocity profile (NULL = 0)                   */
    const double* inlet_T;  /* [ny] K inlet temperature (NULL = T_ref)                       */
    double T_wall[2];       /* K: Dirichlet temperatures at x- and x+ (1D ends, or the
                               D2Q9_D2Q5 side walls of kind LBM_BC_DIRICHLET)             */
    /* two-phase (Sec. 2.3, Sec. 4.4) */
    double rho_l, rho_g;    /* kg/m^3 */
    double nu_l, nu_g;      /* m^2/s, used when visc_mode = 0: nu = nu_g + phi (nu_l - nu_g) */
    double zeta_l, zeta_g;  /* Pa s, used when visc_mode = 1: nu = zeta(phi) / rho(phi)       */
    int visc_mode;
    double sigma, W;        /* N/m, m: beta = 12 sigma / W, kappa = 3 sigma W / 2           */
    double mobility;        /* m^2/s -> tau_phi = M / c_s^2 + dt/2                          */
    int z_collision;        /* LBM_BGK | LBM_MRT                                             */
    int qy_printed;         /* 0: omega_q2 on both q_x and q_y; 1: on q_x only (as printed)  */
    double normal_eps;      /* 1/m: n = 0 where |grad phi| <= normal_eps (<= 0: default)     */
    /* natural convection (App. D): Boussinesq force -rho_ref beta_T (T - T_ref) g added
       to Fb at every node (Eq. buoyancy_force); needs the thermal field */
    double beta_T;          /* 1/K thermal expansion coefficient (0: no buoyancy)           */
    double gravity[2];      /* m/s^2                                                         */
    /* 3D lattices: the z component of the body force; Fb holds x and y.  LBM_D3Q19
       rates are those of Sec. 3 with the 3D basis: e at omega_e, eps at omega_eps,
       the stresses p at 1/tau, q and m at (3/dt)(2/dt - 1/tau)/(3/dt - 1/tau),
       pi at 1/dt (BGK: every non-conserved moment at 1/tau).  LBM_D3Q19_PHASE
       takes the two-phase fields above */
    double Fb_z;            /* N/m^3                                                         */
    /* Relaxation times given directly (s).  tau > 0 replaces nu and tau_T > 0
       replaces alpha, through tau = nu / c_s^2 + dt/2 (Eq. eq_kinematic_viscosity)
       and its thermal analogue: tau for LBM_D2Q9_D2Q5 flow and LBM_D3Q19, tau_T
       for the LBM_D2Q9_D2Q5 temperature and the 1D lattices.  0 = derive them
       from nu and alpha.  The discrete adjoint differentiates with respect to
       these times, so a caller that steps along its gradient passes them here.
       LBM_E_TAU if the resulting time is not above dt/2. */
    double tau, tau_T;
} lbm_params_si;

/* Size in bytes of the device buffer a context with this description needs.
 * Errors: LBM_E_ARG, LBM_E_UNSUPPORTED. */
LBM_API lbm_status lbm_query_bytes(const lbm_desc* desc, size_t* bytes);

/* Create a context on the current HIP device.  desc->dev_buf must hold at
 * least lbm_query_bytes() bytes.  *out is set only on success. */
LBM_API lbm_status lbm_create(const lbm_desc* desc, lbm_ctx** out);

/* Release host resources; enqueued work is not waited for (synchronise the
 * stream first if the buffer is to be reused).  NULL is a no-op. */
LBM_API void lbm_destroy(lbm_ctx* ctx);

/* Compile SI parameters into relaxation rates and kernel constants (Sec. 3:
 * c = dx/dt, c_s^2 = c^2/3 (D1Q2: c^2), tau from nu (or given), tau_T from
 * alpha (or given), tau_phi from M (Eq. source_term_interface text), the
 * dimensional MRT rates of Eq. M_matrix_dim with the omega_q relation of Sec. 3,
 * beta = 12 sigma / W and kappa = 3 sigma W / 2 (Eq. chemical_potential text),
 * qdot = qvol / rho_cp (Eq. forcing_term_g)).  Returns LBM_E_TAU if any
 * relaxation time is not above dt/2, LBM_E_ARG for non-positive dx, dt or
 * densities.  Copies the flux / inlet arrays to the device; the caller keeps
 * ownership of p and of the arrays it points to.  May return the
 * informational LBM_W_FP32_FORCING and LBM_W_MACH bits (parameters set). */
LBM_API lbm_status lbm_set_params_SI(lbm_ctx* ctx, const lbm_params_si* p);

/* 3D lattices: the populations at the equilibria of the given fields, host
 * float64 [batch][nz][ny][nx].  LBM_D3Q19: rho_or_p is the density (kg/m^3,
 * required), phi is ignored.  LBM_D3Q19_PHASE: rho_or_p is the pressure (Pa,
 * NULL = 0), phi the order parameter (required), and (phi u) of the previous
 * step is set to phi u.  ux, uy, uz in m/s (NULL = 0).  Resets the step
 * counter.  Requires lbm_set_params_SI first; LBM_E_ARG for 2D lattices;
 * the informational LBM_W_MACH as for lbm_init_fields. */
LBM_API lbm_status lbm_init_fields3d(lbm_ctx* ctx, const double* rho_or_p, const double* ux,
                                     const double* uy, const double* uz, const double* phi);

/* Set the populations to the equilibria of the given macroscopic fields
 * (host float64 [batch][ny][nx], SI): f_i = f_i^eq of Eq. feq_geral, g_i =
 * g_i^eq of Eq. geq_geral (advective part taken about T_ref), h_i = h_i^eq of
 * Eq. heq_liang and z_i = z_i^eq of Eq. zeq_liang with s_i of Eq. s_i_Liang
 * (the paper gives no initial condition; the equilibrium of the initial fields
 * is the reading taken).  rho_or_p: density (D2Q9_D2Q5, ignored otherwise) or
 * pressure in Pa (PHASE, NULL = 0); ux, uy: m/s (NULL = 0); T: K (thermal and
 * 1D, required there); phi: order parameter (PHASE, required).  The arrays are
 * read before the call returns.  Also resets the step counter and, for PHASE,
 * sets (phi u) of the previous step to phi u.  LBM_E_STATE without
 * lbm_set_params_SI first; LBM_E_ARG for a missing required field; the
 * informational LBM_W_MACH (fields set) when an initial speed exceeds 0.3 dx/dt. */
LBM_API lbm_status lbm_init_fields(lbm_ctx* ctx, const double* rho_or_p, const double* ux,
                           const double* uy, const double* T, const double* phi);

/* Enqueue n time steps (collide + stream + boundary rules, Eq.
 * eq_lattice_boltzmann_geral).  Asynchronous: a non-finite state is reported
 * by lbm_reduce and, with the step count at which it was first seen, by
 * lbm_first_nonfinite_step (see lbm_set_nonfinite_check).  When n is at least twice the graph step count (see
 * lbm_set_graph_steps), runs of that many steps are enqueued as one replay
 * of a HIP graph captured from the same kernel launches (bit-identical
 * results, one launch instead of many on small grids); the remainder and
 * every step whose arguments change with time (the oscillating wall flux)
 * are launched one by one.  No replay is used while desc.hip_stream is being
 * captured by the caller.  A caller that captures lbm_step(n) and replays the
 * graph gets n steps per replay from the buffer the capture started in, so n
 * must be even; lbm_time counts the captured steps once. */
LBM_API lbm_status lbm_step(lbm_ctx* ctx, int n);

/* Failure detection inside lbm_step: every time the step count reaches a
 * multiple of `every` (default 4096; 0 turns the check off), lbm_step
 * enqueues a read-only scan of the state's node values that records the
 * smallest such step count at which any of them was NaN or infinite (no
 * check while the caller captures the stream).  The scan reads the state
 * once, about half a step's memory traffic.  LBM_E_ARG for every < 0. */
LBM_API lbm_status lbm_set_nonfinite_check(lbm_ctx* ctx, int every);

/* The step count at which the check of lbm_set_nonfinite_check first saw a
 * non-finite state since lbm_init_fields / lbm_load_state, or -1 (*step).
 * Synchronous.  Returns LBM_E_NONFINITE (with the step in lbm_last_error)
 * when one was seen, LBM_OK otherwise. */
LBM_API lbm_status lbm_first_nonfinite_step(lbm_ctx* ctx, long long* step);

/* Steps per captured graph used by lbm_step (default 64; 0 disables graph
 * replay; otherwise even, at most 4096).  Graphs are captured lazily on a
 * library-owned stream, one per population-buffer parity, dropped when the
 * count or the parameters change, and released by lbm_destroy.  Not an
 * operation of the paper: a launch-overhead control for small grids.
 * LBM_E_ARG on an odd, negative or too large count. */
LBM_API lbm_status lbm_set_graph_steps(lbm_ctx* ctx, int steps);

/* Kernel choice for LBM_D2Q9_PHASE and LBM_D2Q9_D2Q5 steps.
 *   mode 1: one launch per step (the single-step kernel).
 *   mode 2: pairs of steps run as one launch of a two-step kernel, which
 *           keeps the intermediate state on chip and so moves half the bytes
 *           per step; an odd last step uses the single-step kernel.
 *           LBM_D2Q9_PHASE: a whole row per workgroup when nx is a multiple
 *           of 64 up to 256, otherwise x-tiles of 256 lanes that store 250
 *           columns each and overlap their neighbours by 3 columns per side
 *           (any nx); LBM_E_UNSUPPORTED with LBM_FP32_DEV_ARITH64; ny < 4
 *           uses the single-step kernel.
 *           LBM_D2Q9_D2Q5: x-tiles of 256 lanes that store 252 columns and
 *           overlap by 2 per side; covers flow with temperature (either
 *           thermal set, with or without buoyancy) and every boundary;
 *           LBM_E_UNSUPPORTED for other configurations once
 *           lbm_set_params_SI has been called (before it, such a
 *           configuration steps with the single-step kernel).
 *   mode 3 (LBM_D2Q9_PHASE): every lbm_step call runs as one cooperative
 *           launch (per 16384
 *           steps) of the many-steps kernel: one resident workgroup per
 *           tile, which steps its tile and waits for its neighbouring tiles'
 *           step counters before the next step, so small grids pay no
 *           launch per step.  Needs a split into at most 16 tiles of 512
 *           nodes over all replicas (64 x 8, or nx x 512/nx for nx = 4, 8,
 *           16, 32), LBM_E_UNSUPPORTED otherwise; grids that split into at
 *           most 16 tiles of 128 or 256 nodes run on those.
 *           lbm_step then synchronises the stream before it returns, to read
 *           the kernel's error word: a wait that timed out (a neighbour that
 *           failed, or that other work on the GPU kept from becoming
 *           resident for seconds) gives LBM_E_DEVICE and drops the state.  While the
 *           stream is being captured, steps use the single-step kernel.  The step
 *           counters live in the context's buffer and are reset by
 *           lbm_init_fields and lbm_load_state.  On LBM_D2Q9_D2Q5, mode 3
 *           steps as mode 1.
 *   mode 0 (default): mode 2 where it applies and its workgroups (one per
 *           x-tile and row segment of a replica, the segment length chosen
 *           by a launch-round model when the parameters are set) number at
 *           least 512 and, with x-tiles, at least 90 % of the launched lanes
 *           hold stored columns; else mode 1 (always mode 1 with
 *           LBM_FP32_DEV_ARITH64).
 * The kernels evaluate the same per-node arithmetic in the same order, so
 * the modes agree to the last bit.  Not an operation of the paper: a
 * performance control.  Other lattices ignore it.  LBM_E_ARG on an unknown
 * mode. */
LBM_API lbm_status lbm_set_step_fusion(lbm_ctx* ctx, int mode);

/* Macroscopic fields of the current state, evaluated in FP64 from the stored
 * populations: rho = sum f_i (Eq. zero_moment_f), u = (sum c_i f_i + dt F/2) /
 * rho (Eq. first_moment_f), T = sum g_i + dt qdot/2 (Eq. zero_moment_g); for
 * the two-phase models phi = sum h_i (Eq. zero_moment_h), rho linear in phi
 * (text after Eq. zero_moment_h), u from the z_i (Eq. u_Liang), p (Eq.
 * p_Liang) and mu (Eq. chemical_potential).  mask selects fields; out receives
 * them in bit order, each [batch][ny][nx] float64 (caller-owned, popcount(mask)
 * x batch x ny x nx doubles):
 *   LBM_M_RHO (density), LBM_M_P (PHASE pressure, Pa), LBM_M_UX, LBM_M_UY (m/s),
 *   LBM_M_T (K), LBM_M_PHI, LBM_M_MU (chemical potential, Pa), LBM_M_UZ (m/s,
 *   3D lattices).  LBM_D3Q19_PHASE offers RHO, P, UX, UY, UZ, PHI and MU.
 * out_on_device != 0: out is a device pointer (written on the stream,
 * asynchronous); otherwise a host pointer (synchronous). */
enum { LBM_M_RHO = 1, LBM_M_P = 2, LBM_M_UX = 4, LBM_M_UY = 8, LBM_M_T = 16,
       LBM_M_PHI = 32, LBM_M_MU = 64, LBM_M_UZ = 128 };
LBM_API lbm_status lbm_macros(lbm_ctx* ctx, unsigned mask, double* out, int out_on_device);

/* FP64 global sums per replica, deterministic (fixed-order two-pass
 * reduction): the conserved totals of the method -- the mass sum rho (Eq.
 * zero_moment_f, conserved by the collision of Eq. colisao_MRT), the order
 * parameter sum phi (Eq. zero_moment_h, conserved by the conservative
 * Allen-Cahn equation, Eq. Allen_cahn) and the energy sum T (Eq.
 * zero_moment_g) -- evaluated from the stored populations.  out (host,
 * caller-owned, popcount(mask) x batch doubles) receives, per selected bit in
 * bit order, batch values:
 *   LBM_R_MASS (sum of rho, kg/m^3 * nodes), LBM_R_PHASE (sum of phi),
 *   LBM_R_ENERGY (sum of T, K * nodes), LBM_R_NONFINITE (count of NaN/Inf
 *   populations).  Synchronous.  Returns LBM_E_NONFINITE when any population
 *   is not finite (out is still filled). */
enum { LBM_R_MASS = 1, LBM_R_PHASE = 2, LBM_R_ENERGY = 4, LBM_R_NONFINITE = 8 };
LBM_API lbm_status lbm_reduce(lbm_ctx* ctx, unsigned mask, double* out);

/* lbm_reduce for callers that cannot allocate device memory or take a
 * workspace at the call (code under stream capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and the same results,
 * but the FP64 partials and per-replica sums live in a static device array
 * of the library (8.4 MB per GPU, held until the process ends) instead of
 * the context's buffer, and the call makes no allocation of any kind.  At
 * most 1024 replicas (LBM_E_ARG beyond).  Calls that overlap on one GPU share
 * that array and race; calls on one stream are ordered.  Synchronous; returns
 * LBM_E_NONFINITE like lbm_reduce. */
LBM_API lbm_status lbm_reduce_noalloc(lbm_ctx* ctx, unsigned mask, double* out);

/* Heated-channel diagnostics of replica 0 (LBM_D2Q9_D2Q5 with flow and
 * thermal): per column the mixing-cup temperature Tb = sum(u T)/sum(u), the
 * wall temperature Tw = mean of the two wall-adjacent nodes + q'' dx/(2k), and
 * Nu = q'' 2H / (k (Tw - Tb)), k = rho_cp alpha, H = ny dx (the paper reports
 * Nu without a formula; this is the reading used).  Any output may be NULL;
 * nu_mean is the mean of Nu over columns x >= x_dev; T_out = Tb[nx-1].
 * Synchronous. */
LBM_API lbm_status lbm_nusselt(lbm_ctx* ctx, int x_dev, double* Tb, double* Tw, double* Nu,
                       double* nu_mean, double* T_out);

/* ---- discrete adjoint of the heated channel --------------------------------
 * Objective (the paper gives no gradients; this is the differentiated quantity):
 * J = w_tout * T_out + w_nu * mean_{x >= x_dev} Nu(x) at the last recorded step,
 * with T_out and Nu as in lbm_nusselt.  Parameters: the wall-flux profile
 * flux[nx] (both walls) and the relaxation times tau (momentum) and tau_T
 * (temperature), which set nu = (tau - dt/2) c_s^2 and alpha = (tau_T - dt/2) c_s^2.
 * Supported for LBM_D2Q9_D2Q5 with flow and thermal populations, inlet/outlet
 * in x, walls in y, batch 1. */
typedef struct {
    int x_dev;              /* first column of the Nusselt average                          */
    double w_tout, w_nu;    /* weights of the two terms                                     */
} lbm_objective;

/* Bytes of the caller-owned device work buffer lbm_record needs for nsteps
 * steps with a checkpoint every ckpt_every steps: the checkpoints, a
 * recomputation tape of ckpt_every + 1 states, two adjoint states and the FP64
 * accumulators. */
LBM_API lbm_status lbm_query_record_bytes(const lbm_ctx* ctx, int nsteps, int ckpt_every,
                                          size_t* bytes);

/* Advance nsteps from the current state (as lbm_step), saving the state every
 * ckpt_every steps into work (device memory of lbm_query_record_bytes bytes,
 * 256-byte aligned, kept alive until lbm_grad), and return J (synchronous).
 * The context then holds the final state. */
LBM_API lbm_status lbm_record(lbm_ctx* ctx, int nsteps, int ckpt_every,
                              const lbm_objective* obj, void* work, size_t work_bytes,
                              double* J);

/* Reverse sweep of the last lbm_record: recompute each checkpoint segment
 * (the forward step kernel writes the tape), then apply the hand-written
 * discrete adjoint step backwards.  Outputs dL/dJ * dJ/dflux[nx] (per W/m^2)
 * and dL/dJ * dJ/dtau[2] = (d/dtau, d/dtau_T) (per second), accumulated in
 * FP64 in a fixed order (deterministic).  Synchronous.  The context keeps the
 * final state. */
LBM_API lbm_status lbm_grad(lbm_ctx* ctx, double dL_dJ, double* dJ_dflux, double* dJ_dtau);

/* Number of steps taken since lbm_init_fields / lbm_load_state. */
LBM_API long long lbm_time(const lbm_ctx* ctx);

/* Serialise the state (populations, (phi u), step counter, a hash of the
 * description and parameters) to host memory: every node value of the state in
 * the device layout's order, without its padding, so equal states give equal
 * blobs.
 * Call with host = NULL to get the size in *bytes.  Synchronous. */
LBM_API lbm_status lbm_save_state(lbm_ctx* ctx, void* host, size_t* bytes);

/* Restore a state written by lbm_save_state for an identical description
 * and parameters; LBM_E_STATE on size, magic or hash mismatch. */
LBM_API lbm_status lbm_load_state(lbm_ctx* ctx, const void* host, size_t bytes);

/* Text of the last error on this context (never NULL). */
LBM_API const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */

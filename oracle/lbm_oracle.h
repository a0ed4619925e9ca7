/*
 * lbm_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct FP64 CPU implementation of the dimensional
 * lattice Boltzmann method (arXiv 2302.04120): every quantity in SI units,
 * no conversion to lattice units (Sec. 3).  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the HIP library; the two never include
 * or link each other.
 *
 * Storage convention: populations are kept in full (no reference-state
 * deviations), as pre-collision ("post-streaming") values, layout [q][ny][nx]
 * with x fastest.  One time step = macros -> equilibria/sources -> collision
 * -> streaming -> boundary substitution (Sec. 2.1, Eq. eq_lattice_boltzmann_geral
 * and the text following Eq. colisao_MRT).
 *
 * Pins: the CPU tests hold these functions to closed forms, printed values,
 * invariants and brute force.  Parity unpinned (no closed form or printed
 * value exists; only the kernel-oracle comparison holds them):
 *   - orc_chan_* with flux_amp != 0: the mean Nu of the oscillating flux
 *     (the flux modulation itself is pinned by the exact wall energy input);
 *   - orc_phase_*: the magnitude of the spurious currents around a bubble
 *     (their square symmetry is pinned by the mirror and transpose tests);
 *   - orc_chan_adjoint: the gradients with respect to the relaxation times
 *     (held by central differences of the oracle's own forward run and by
 *     the hand-written FP64 adjoint, not by an independent value).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- 1D thermal (D1Q2 / D1Q3), wet-node Dirichlet ends -------- */
/* Sec. 2.2 (Eq. eq_lattice_boltzmann_BGK_T, forcing_term_g, geq_geral,
 * zero_moment_g); wet-node Dirichlet of App. B (Eq. BCs_1D_advection_diffusion)
 * with the half-source term of Eq. zero_moment_g.  q = 2 or 3.
 * T_init[n] (K) in, T_out[n] (K) out.  Returns 0 or a negative error. */
int orc_d1_run(int q, int n, double dx, double dt, double alpha, double qdot,
               double u, double T0, double TL, const double* T_init,
               long nsteps, double* T_out);

/* ---------------- matrices (Sec. 2.1 Eq. M_matrix, Sec. 3 Eq. M_matrix_dim) - */
/* Writes the dimensional D2Q9 transformation matrix and its numerical inverse
 * (row-major 9x9). */
void orc_mdim(double c, double* M_out, double* Minv_out);

/* ---------------- single-phase channel: D2Q9 flow + optional D2Q5 thermal --- */
typedef struct {
    int nx, ny;
    int bc_x;          /* 0 periodic, 1 velocity inlet (x-) + pressure outlet (x+),
                          2 no-slip walls at fixed temperatures Tw_x (App. D)      */
    int bc_y;          /* 0 periodic, 1 halfway walls at y- and y+, 2 halfway wall at
                          y- and a symmetry plane at y+ (Eq. simetria)               */
    double dx, dt;
    /* flow */
    int flow;          /* 0 frozen (populations not updated), 1 D2Q9 */
    int flow_mrt;      /* 0 BGK, 1 dimensional MRT */
    double rho_ref, nu, omega_e, omega_eps;  /* omega_* in 1/s */
    double Fx, Fy;     /* body force, N/m^3 */
    /* thermal */
    int thermal;       /* 0 none, 1 D2Q5, 2 D2Q9 */
    int thermal_mrt;   /* 0 BGK; 1 MRT: D2Q5 two-rate (j at 1/tau_T, e and pxx at
                          1/dt), D2Q9 Lambda_T,dim of Sec. 3 (j at 1/tau_T, the
                          rest at 1/dt)                                           */
    double alpha, rho_cp, qdot, T_ref;       /* qdot in K/s */
    double flux_amp, flux_omega;              /* q''(x,t) = flux[x](1 + amp sin(omega t)) */
    double Tw_x[2];    /* bc_x == 2: wall temperatures at x- and x+ (K)               */
    double buoy[2];    /* Boussinesq force per kelvin of T - T_ref, -rho_ref beta g
                          (Eq. buoyancy_force), N/m^3/K; 0 disables                  */
} orc_chan_params;

typedef struct orc_chan orc_chan;
orc_chan* orc_chan_create(const orc_chan_params* p, const double* flux /*[nx] W/m^2*/,
                          const double* inlet_u /*[ny] m/s*/, const double* inlet_T /*[ny] K*/);
void orc_chan_destroy(orc_chan* s);
/* equilibrium populations from macros [ny][nx] (T may be NULL when thermal==0) */
void orc_chan_init(orc_chan* s, const double* rho, const double* ux, const double* uy,
                   const double* T);
void orc_chan_step(orc_chan* s, long nsteps);
/* macros of the current (pre-collision) state; any pointer may be NULL */
void orc_chan_macros(const orc_chan* s, double* rho, double* ux, double* uy, double* T);
long orc_chan_time(const orc_chan* s);
/* raw state: f[9][ny][nx] then g[5 or 9][ny][nx]; plus the time index */
void orc_chan_get_state(const orc_chan* s, double* f, double* g);
void orc_chan_set_state(orc_chan* s, const double* f, const double* g, long t);
/* replace the wall flux profile / inlet temperature (W/m^2 per column) */
void orc_chan_set_flux(orc_chan* s, const double* flux);
void orc_chan_set_tau(orc_chan* s, double nu, double alpha);

/* Diagnostics of the channel case (FP64): per-column bulk (mixing-cup)
 * temperature, wall temperature and local Nusselt number; see the Nu
 * definition documented in orc_chan_objective.  k = rho_cp * alpha. */
void orc_chan_nusselt(const orc_chan* s, double* Tb, double* Tw, double* Nu);
/* J = mixing-cup outlet temperature + mean Nu over x >= x_dev (column index) */
double orc_chan_objective(const orc_chan* s, int x_dev, double w_tout, double w_nu);

/* FP64 discrete adjoint of orc_chan over nsteps from the current state,
 * checkpointing every ckpt steps and recomputing within each segment.
 * Objective as orc_chan_objective at the final state.  Outputs dJ/dflux[nx],
 * dJ/dtau[2] = (dJ/dtau_nu, dJ/dtau_T), and J.  The object is left at the
 * final state.  Returns 0 or negative. */
int orc_chan_adjoint(orc_chan* s, long nsteps, int ckpt, int x_dev, double w_tout,
                     double w_nu, double* J, double* dJ_dflux, double* dJ_dtau);

/* ---------------- two-phase: conservative Allen-Cahn h + pressure z -------- */
typedef struct {
    int nx, ny;
    int bc_y;          /* 0 periodic, 1 halfway walls (x is always periodic) */
    double dx, dt;
    double rho_l, rho_g, nu_l, nu_g, zeta_l, zeta_g;
    int visc_mode;     /* 0: nu = nu_g + phi(nu_l-nu_g); 1: nu = zeta(phi)/rho(phi) */
    double sigma, W, M;
    double Fbx, Fby;
    int z_mrt;         /* 0 BGK, 1 dimensional MRT */
    int qy_printed;    /* 0: omega_q2 on both q_x and q_y; 1: on q_x only */
    double normal_eps; /* |grad phi| at or below this (1/m) gives n = 0 */
} orc_phase_params;

typedef struct orc_phase orc_phase;
orc_phase* orc_phase_create(const orc_phase_params* p);
void orc_phase_destroy(orc_phase* s);
void orc_phase_init(orc_phase* s, const double* phi, const double* p, const double* ux,
                    const double* uy);
void orc_phase_step(orc_phase* s, long nsteps);
/* phi, rho, p, ux, uy, mu of the current state; any may be NULL */
void orc_phase_macros(const orc_phase* s, double* phi, double* rho, double* p, double* ux,
                      double* uy, double* mu);
/* grad phi (x, y) and laplacian of phi by the stencils of Sec. 2.3 */
void orc_phase_gradients(const orc_phase* s, double* gx, double* gy, double* lap);
void orc_phase_get_state(const orc_phase* s, double* h, double* z, double* phiu);
void orc_phase_set_state(orc_phase* s, const double* h, const double* z, const double* phiu);

/* ---- 3D momentum: D3Q19 with the dimensional MRT (Sec. 3 in three dimensions) ---- */
typedef struct {
    int nx, ny, nz;
    int bc_x, bc_y, bc_z; /* per axis: 0 periodic, 1 halfway walls on both sides */
    double dx, dt;
    int mrt;           /* 0 BGK, 1 dimensional MRT */
    double rho_ref, nu, omega_e, omega_eps;  /* omega_* in 1/s (<= 0: 1/dt) */
    double F[3];       /* body force, N/m^3 */
} orc_d3_params;

typedef struct orc_d3 orc_d3;
/* the dimensional D3Q19 moment matrix (rows scaled by c^degree) and its inverse */
void orc_d3_mdim(double c, double* M /*[19*19]*/, double* Minv /*[19*19]*/);
orc_d3* orc_d3_create(const orc_d3_params* p);
void orc_d3_destroy(orc_d3* s);
/* equilibrium populations from macros, arrays [nz][ny][nx] */
void orc_d3_init(orc_d3* s, const double* rho, const double* ux, const double* uy,
                 const double* uz);
void orc_d3_step(orc_d3* s, long nsteps);
void orc_d3_macros(const orc_d3* s, double* rho, double* ux, double* uy, double* uz);
void orc_d3_get_state(const orc_d3* s, double* f /*[19][nz][ny][nx]*/);
void orc_d3_set_state(orc_d3* s, const double* f /*[19][nz][ny][nx]*/);

/* ---- 3D two-phase model (Sec. 2.3 on D3Q19, z_i with the dimensional MRT) ---- */
typedef struct {
    int nx, ny, nz;
    int bc_x, bc_y, bc_z;   /* per axis: 0 periodic, 1 halfway walls on both sides */
    double dx, dt;
    double rho_l, rho_g, nu_l, nu_g, zeta_l, zeta_g;
    int visc_mode;          /* 0: nu linear in phi; 1: zeta linear, nu = zeta / rho */
    double sigma, W, M;     /* N/m, m, m^2/s */
    double Fb[3];           /* N/m^3 */
    int z_mrt;              /* 0 BGK, 1 dimensional MRT */
    double normal_eps;      /* 1/m: n = 0 where |grad phi| <= normal_eps */
} orc_p3_params;

typedef struct orc_p3 orc_p3;
orc_p3* orc_p3_create(const orc_p3_params* p);
void orc_p3_destroy(orc_p3* s);
/* equilibria of phi, pressure p (Pa) and u (m/s), arrays [nz][ny][nx] */
void orc_p3_init(orc_p3* s, const double* phi, const double* p, const double* ux,
                 const double* uy, const double* uz);
void orc_p3_step(orc_p3* s, long nsteps);
void orc_p3_macros(const orc_p3* s, double* phi, double* rho, double* p, double* ux,
                   double* uy, double* uz, double* mu);
void orc_p3_gradients(const orc_p3* s, double* gx, double* gy, double* gz, double* lap);
void orc_p3_get_state(const orc_p3* s, double* h /*[19]*/, double* z /*[19]*/,
                      double* phiu /*[3]*/);
void orc_p3_set_state(orc_p3* s, const double* h /*[19]*/, const double* z /*[19]*/,
                      const double* phiu /*[3]*/);

#ifdef __cplusplus
}
#endif
#endif

/* Drives every entry point of the FP64 oracle on small grids with every
 * boundary kind, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only).  Exit status 0 when every call
 * succeeded and every output is finite; the sanitizers abort on any invalid
 * access, leak or undefined operation. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

static int finite_all(const double* a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                \
        }                                                            \
    } while (0)

static int d1(void) {
    double T0[11], T1[11];
    for (int i = 0; i < 11; ++i) T0[i] = 300.0 + i;
    for (int q = 2; q <= 3; ++q) {
        CHECK(orc_d1_run(q, 11, 1e-3, 1e-2, 1e-5, 10.0, 0.0, 300.0, 310.0, T0, 50, T1) == 0);
        CHECK(finite_all(T1, 11));
    }
    double M[81], Mi[81];
    orc_mdim(2.0, M, Mi);
    CHECK(finite_all(M, 81) && finite_all(Mi, 81));
    return 0;
}

static int chan(int bc_x, int bc_y, int thermal) {
    const int nx = 9, ny = 5, N = nx * ny;
    orc_chan_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx; p.ny = ny; p.bc_x = bc_x; p.bc_y = bc_y;
    p.dx = 1e-4; p.dt = 1e-3; p.flow = 1; p.flow_mrt = 1;
    p.rho_ref = 1000.0; p.nu = 1e-6; p.omega_e = 1.1e3; p.omega_eps = 0.9e3;
    p.Fx = 1.0; p.thermal = thermal; p.thermal_mrt = 1;
    p.alpha = 1.5e-7; p.rho_cp = 4.2e6; p.qdot = 1.0; p.T_ref = 300.0;
    p.flux_amp = 0.5; p.flux_omega = 3.0; p.Tw_x[0] = 305.0; p.Tw_x[1] = 295.0;
    p.buoy[1] = bc_x == 2 ? 0.5 : 0.0;  /* Boussinesq force with the heated side walls */
    double flux[9], uin[5], Tin[5];
    for (int x = 0; x < nx; ++x) flux[x] = 1e3 * (1 + x % 3);
    for (int y = 0; y < ny; ++y) { uin[y] = 1e-5 * (1 + y); Tin[y] = 300.0; }
    orc_chan* s = orc_chan_create(&p, flux, uin, Tin);
    CHECK(s != NULL);
    double* buf = calloc(40 * (size_t)N, sizeof(double));
    double *rho = buf, *ux = buf + N, *uy = buf + 2 * N, *T = buf + 3 * N;
    for (int i = 0; i < N; ++i) { rho[i] = 1000.0; ux[i] = 1e-5; uy[i] = 0.0; T[i] = 300.0 + i % 3; }
    orc_chan_init(s, rho, ux, uy, thermal ? T : NULL);
    orc_chan_step(s, 20);
    orc_chan_macros(s, rho, ux, uy, T);
    CHECK(finite_all(buf, 4 * (size_t)N));
    double* f = buf + 4 * N;
    double* g = buf + 13 * N;
    orc_chan_get_state(s, f, g);
    orc_chan_set_state(s, f, g, orc_chan_time(s));
    orc_chan_set_flux(s, flux);
    orc_chan_set_tau(s, 1.2e-6, 1.6e-7);
    if (thermal) {
        double Tb[9], Tw[9], Nu[9], J = 0, dq[9], dt[2];
        orc_chan_nusselt(s, Tb, Tw, Nu);
        (void)orc_chan_objective(s, nx / 2, 1.0, 1.0);
        const int rc = orc_chan_adjoint(s, 30, 7, nx / 2, 1.0, 1.0, &J, dq, dt);
        if (bc_x == 1 && bc_y == 1 && thermal == 1) {
            CHECK(rc == 0);
            CHECK(isfinite(J) && finite_all(dq, 9) && finite_all(dt, 2));
        } else {
            CHECK(rc == -2);  /* the adjoint covers the heated channel only */
        }
    }
    orc_chan_destroy(s);
    free(buf);
    return 0;
}

static int phase(int bc_y, int visc_mode) {
    const int nx = 7, ny = 6, N = nx * ny;
    orc_phase_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx; p.ny = ny; p.bc_y = bc_y; p.dx = 5e-6; p.dt = 1e-7;
    p.rho_l = 1000.0; p.rho_g = 1.0; p.nu_l = 1e-6; p.nu_g = 1e-5;
    p.zeta_l = 1e-3; p.zeta_g = 1e-5; p.visc_mode = visc_mode;
    p.sigma = 0.07; p.W = 2e-5; p.M = 1e-5; p.Fbx = 10.0; p.z_mrt = 1; p.normal_eps = 1.0;
    orc_phase* s = orc_phase_create(&p);
    CHECK(s != NULL);
    double* buf = calloc(40 * (size_t)N, sizeof(double));
    double *phi = buf, *pr = buf + N, *ux = buf + 2 * N, *uy = buf + 3 * N;
    for (int i = 0; i < N; ++i) { phi[i] = 0.3 + 0.05 * (i % 7); pr[i] = 5.0; ux[i] = 1e-4; uy[i] = -1e-4; }
    orc_phase_init(s, phi, pr, ux, uy);
    orc_phase_step(s, 15);
    orc_phase_macros(s, phi, buf + 4 * N, pr, ux, uy, buf + 5 * N);
    CHECK(finite_all(buf, 6 * (size_t)N));
    orc_phase_gradients(s, buf, buf + N, buf + 2 * N);
    CHECK(finite_all(buf, 3 * (size_t)N));
    double *h = buf + 6 * N, *z = buf + 15 * N, *pu = buf + 24 * N;
    orc_phase_get_state(s, h, z, pu);
    orc_phase_set_state(s, h, z, pu);
    orc_phase_step(s, 1);
    orc_phase_destroy(s);
    free(buf);
    return 0;
}

static int d3(int bc) {
    const int nx = 5, ny = 4, nz = 3, N = nx * ny * nz;
    orc_d3_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx; p.ny = ny; p.nz = nz; p.bc_x = bc; p.bc_y = 1 - bc; p.bc_z = bc;
    p.dx = 1e-4; p.dt = 1e-3; p.mrt = 1; p.rho_ref = 1000.0; p.nu = 1e-6;
    p.F[0] = 1.0; p.F[2] = -0.5;
    double M[361], Mi[361];
    orc_d3_mdim(0.1, M, Mi);
    CHECK(finite_all(M, 361) && finite_all(Mi, 361));
    orc_d3* s = orc_d3_create(&p);
    CHECK(s != NULL);
    double* buf = calloc(24 * (size_t)N, sizeof(double));
    for (int i = 0; i < N; ++i) { buf[i] = 1000.0; buf[N + i] = 1e-4; }
    orc_d3_init(s, buf, buf + N, buf + 2 * N, buf + 3 * N);
    orc_d3_step(s, 10);
    orc_d3_macros(s, buf, buf + N, buf + 2 * N, buf + 3 * N);
    CHECK(finite_all(buf, 4 * (size_t)N));
    orc_d3_get_state(s, buf + 4 * N);
    orc_d3_set_state(s, buf + 4 * N);
    orc_d3_step(s, 1);
    orc_d3_destroy(s);
    free(buf);
    return 0;
}

static int p3(int bc) {
    const int nx = 5, ny = 4, nz = 3, N = nx * ny * nz;
    orc_p3_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx; p.ny = ny; p.nz = nz; p.bc_x = bc; p.bc_y = 1 - bc; p.bc_z = bc;
    p.dx = 5e-6; p.dt = 1e-7; p.rho_l = 1000.0; p.rho_g = 1.0; p.nu_l = 1e-6; p.nu_g = 1e-5;
    p.zeta_l = 1e-3; p.zeta_g = 1e-5; p.sigma = 0.07; p.W = 2e-5; p.M = 1e-5;
    p.Fb[1] = 5.0; p.z_mrt = 1; p.normal_eps = 1.0;
    orc_p3* s = orc_p3_create(&p);
    CHECK(s != NULL);
    double* buf = calloc(48 * (size_t)N, sizeof(double));
    for (int i = 0; i < N; ++i) { buf[i] = 0.2 + 0.1 * (i % 5); buf[N + i] = 3.0; buf[2 * N + i] = 1e-4; }
    orc_p3_init(s, buf, buf + N, buf + 2 * N, buf + 3 * N, buf + 4 * N);
    orc_p3_step(s, 8);
    orc_p3_macros(s, buf, buf + N, buf + 2 * N, buf + 3 * N, buf + 4 * N, buf + 5 * N, buf + 6 * N);
    CHECK(finite_all(buf, 7 * (size_t)N));
    orc_p3_gradients(s, buf, buf + N, buf + 2 * N, buf + 3 * N);
    CHECK(finite_all(buf, 4 * (size_t)N));
    orc_p3_get_state(s, buf + 7 * N, buf + 26 * N, buf + 45 * N);
    orc_p3_set_state(s, buf + 7 * N, buf + 26 * N, buf + 45 * N);
    orc_p3_step(s, 1);
    orc_p3_destroy(s);
    free(buf);
    return 0;
}

int main(void) {
    if (d1()) return 1;
    for (int bx = 0; bx <= 2; ++bx)
        for (int by = 0; by <= 2; ++by)
            for (int th = 0; th <= 2; ++th)
                if (chan(bx, by, th)) return 1;
    for (int by = 0; by <= 1; ++by)
        for (int vm = 0; vm <= 1; ++vm)
            if (phase(by, vm)) return 1;
    for (int bc = 0; bc <= 1; ++bc)
        if (d3(bc) || p3(bc)) return 1;
    printf("oracle sanitizer driver: all entry points ran\n");
    return 0;
}

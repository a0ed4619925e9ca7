// HIP kernels of the dimensional LBM hot path for gfx950 (CDNA4, wave64).
//
// Data layout: structure of arrays, one plane per population, plane index
// i * P + (b * ny + y) * nx + x (x fastest, P a multiple of 64 elements).
// The stored state is the pre-collision ("post-streaming") population set;
// each step reads a node's own populations (coalesced), collides in
// registers and pushes the post-collision values to x + e_i in the other
// buffer.  Populations whose destination lies outside the domain are turned
// back into the node by the boundary rule of that side, so every slot of the
// next buffer is written exactly once and no two threads write the same slot.
//
// All arithmetic is in lattice-normalised form (velocities / c, forces
// F dt^2 / dx, rates Lambda dt).  The dimensional MRT of Sec. 3 multiplies
// the rows of the lattice matrix by c^order and its inverse's columns by
// c^-order; a diagonal relaxation commutes with that scaling, so the
// post-collision populations are the same in either form.
#include "lbm_device.h"

#include <cmath>
#include <type_traits>

namespace lbm {
namespace {

template <typename S>
__global__ __launch_bounds__(256) void k_chan_step(ChanK k, const S* __restrict__ fc,
                                                   S* __restrict__ fn, const S* __restrict__ gc,
                                                   S* __restrict__ gn, const S* __restrict__ qw,
                                                   const S* __restrict__ uin,
                                                   const S* __restrict__ tin, S mod) {
    using C = S;
    const int nx = k.nx, ny = k.ny;
    const int gx = (nx + 63) / 64, gy = (ny + 3) / 4;
    int tile;
    if (!xcd_tile(gx * gy * k.batch, tile)) return;
    const int b = tile / (gx * gy), r = tile - b * gx * gy;
    const int x = (r % gx) * 64 + threadIdx.x;
    const int y = (r / gx) * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const long long P = k.P;
    const long long base = (long long)b * ny * nx;
    const long long n = base + (long long)y * nx + x;
    const C rho_ref = C(k.rho_ref), ftx = C(k.Ft[0]), fty = C(k.Ft[1]);

    C d[9], drho, rho, ux, uy;
    chan_flow_macros<C, S>(fc, P, n, rho_ref, ftx, fty, d, drho, rho, ux, uy);

    // ---- momentum collision (Eq. colisao_MRT or Eq. eq_lattice_boltzmann_BGK)
    C ds[9];
    if (k.flow) {
        const C uu = ux * ux + uy * uy;
        C neq[9], fh[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const C eu = C(EX[i]) * ux + C(EY[i]) * uy;
            // deviation of Eq. feq_geral from w_i rho_ref
            const C feq = wgt<C>(i) * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu));
            neq[i] = d[i] - feq;
            // dt * Guo term of Eq. forcing_term (without its prefactor)
            fh[i] = wgt<C>(i) * ((C(3) * (C(EX[i]) - ux) + C(9) * eu * C(EX[i])) * ftx +
                                 (C(3) * (C(EY[i]) - uy) + C(9) * eu * C(EY[i])) * fty);
        }
        if (k.flow_mrt) {
            C mn[9], mf[9], dm[9], dv[9];
            moments9(neq, mn);
            moments9(fh, mf);
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const C L = C(k.Lf[q]);
                dm[q] = -L * mn[q] + (C(1) - C(0.5) * L) * mf[q];
            }
            inverse9(dm, dv);
#pragma unroll
            for (int i = 0; i < 9; ++i) ds[i] = d[i] + dv[i];
        } else {
            const C L = C(k.Lf[7]);
#pragma unroll
            for (int i = 0; i < 9; ++i) ds[i] = d[i] - L * neq[i] + (C(1) - C(0.5) * L) * fh[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) ds[i] = d[i];
    }

    // ---- temperature collision (Sec. 2.2), advective part built on T - T_ref
    C es[5];
    if (k.thermal) {
        C e[5], neq[5], m[5], dm[5], dv[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) e[i] = C(gc[i * P + n]);
        const C qdt = C(k.qdt);
        const C th = (e[0] + (e[1] + e[3]) + (e[2] + e[4])) + C(0.5) * qdt;  // Eq. zero_moment_g
#pragma unroll
        for (int i = 0; i < 5; ++i)
            neq[i] = e[i] - wgt5<C>(i) * th * (C(1) + C(3) * (C(EX5[i]) * ux + C(EY5[i]) * uy));
        moments5(neq, m);
        // moments of the source w_i qdot dt: qdt (1, 0, 0, -2/3, 0)
        const C ms[5] = {qdt, C(0), C(0), C(-2) / C(3) * qdt, C(0)};
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const C L = C(k.Lt[q]);
            dm[q] = -L * m[q] + (C(1) - C(0.5) * L) * ms[q];
        }
        inverse5(dm, dv);
#pragma unroll
        for (int i = 0; i < 5; ++i) es[i] = e[i] + dv[i];
    }

    // ---- outlet wall velocity: 1.5 u(x_b) - 0.5 u(x_b - 1) at time t
    C uwx = C(0), uwy = C(0);
    const bool outlet = k.bcx && x == nx - 1;
    if (k.flow && outlet) {
        C d2[9], dr2, r2, ux2, uy2;
        chan_flow_macros<C, S>(fc, P, n - 1, rho_ref, ftx, fty, d2, dr2, r2, ux2, uy2);
        uwx = C(1.5) * ux - C(0.5) * ux2;
        uwy = C(1.5) * uy - C(0.5) * uy2;
    }

    // ---- streaming with boundary substitution (a frozen flow keeps its populations)
    if (!k.flow) {
#pragma unroll
        for (int i = 0; i < 9; ++i) fn[i * P + n] = S(d[i]);
    } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int tx = x + EX[i], ty = y + EY[i];
        const bool outy = k.bcy && (ty < 0 || ty >= ny);
        const bool outx = k.bcx && (tx < 0 || tx >= nx);
        if (!outy && !outx) {
            tx = wrap(tx, nx);
            ty = wrap(ty, ny);
            fn[i * P + base + (long long)ty * nx + tx] = S(ds[i]);
        } else {
            C v;
            if (outy) {
                v = ds[i];  // halfway bounce-back, Eq. BB_vel with u_w = 0
            } else if (tx < 0) {
                // moving-wall bounce-back with the inlet profile, Eq. BB_vel
                v = ds[i] - C(6) * wgt<C>(i) * rho_ref * (C(EX[i]) * C(uin[y]));
            } else {
                // anti-bounce-back pressure outlet, Eq. anti_BB_vel, rho_w = rho_ref
                const C eu = C(EX[i]) * uwx + C(EY[i]) * uwy;
                v = -ds[i] + C(2) * wgt<C>(i) * rho_ref *
                                 (C(4.5) * eu * eu - C(1.5) * (uwx * uwx + uwy * uwy));
            }
            fn[OPP[i] * P + n] = S(v);
        }
    }
    }
    if (k.thermal) {
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            int tx = x + EX5[i], ty = y + EY5[i];
            const bool outy = k.bcy && (ty < 0 || ty >= ny);
            const bool outx = k.bcx && (tx < 0 || tx >= nx);
            if (!outy && !outx) {
                tx = wrap(tx, nx);
                ty = wrap(ty, ny);
                gn[i * P + base + (long long)ty * nx + tx] = S(es[i]);
            } else if (outy) {
                // prescribed flux, Eq. BB_T with lambda = 1 on D2Q5
                gn[OPP5[i] * P + n] = S(es[i] + C(qw[x]) * C(mod));
            } else if (tx < 0) {
                // anti-bounce-back Dirichlet inlet, Eq. anti_BB_T (deviation form)
                gn[OPP5[i] * P + n] = S(-es[i] + C(2) * wgt5<C>(i) * C(tin[y]));
            } else {
                // first-order extrapolation outlet: the incoming population keeps
                // the value streamed into x_b - 1, i.e. this node's own post-collision
                gn[OPP5[i] * P + n] = S(es[OPP5[i]]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Two-phase step: conservative Allen-Cahn h_i (BGK) + pressure z_i (MRT/BGK)
// Tile of 64 x TY nodes per block; phi of the tile and a one-node ring in LDS.
// Buffer planes: 0-8 h_i, 9-17 z_i, 18 low part of h_0 (FP32 storage only).
// ---------------------------------------------------------------------------

#ifndef LBM_PHASE_TY
#define LBM_PHASE_TY 8
#endif
// optional occupancy target (waves per SIMD) for the step kernel; 0 = compiler's choice
#ifndef LBM_PHASE_WPE
#define LBM_PHASE_WPE 0
#endif
#if LBM_PHASE_WPE > 0
#define LBM_PHASE_OCC __attribute__((amdgpu_waves_per_eu(LBM_PHASE_WPE)))
#else
#define LBM_PHASE_OCC
#endif
constexpr int TX = 64, TY = LBM_PHASE_TY;
// LDS reserved by each FP32 step workgroup beyond its own 2.6 KB: it holds
// residency at two 512-thread workgroups per CU (4 waves per SIMD).  With
// more waves resident, more of the 42 population streams per wave are open
// in DRAM at once and the step runs slower (67M-node bubble batch: 2.82 ms
// at 8 waves per SIMD, 2.56 ms at 4).  The FP64 kernel's register use
// already gives 4 waves per SIMD.
constexpr unsigned kPhaseLdsReserve = 61440;
static_assert(2 * (TX + 2) + 2 * TY <= TX * TY, "the ring must fit in one pass of the block");

template <typename S, typename C>
__device__ __forceinline__ C node_phi(const S* __restrict__ h, const S* __restrict__ hlo,
                                      long long P, long long n) {
    C a = C(h[n]);
    if (hlo) a += C(hlo[n]);
    C s = (C(h[P + n]) + C(h[3 * P + n])) + (C(h[2 * P + n]) + C(h[4 * P + n]));
    s += (C(h[5 * P + n]) + C(h[7 * P + n])) + (C(h[6 * P + n]) + C(h[8 * P + n]));
    return a + s;  // Eq. zero_moment_h
}

template <typename S, typename C, bool MACROS>
__global__ __launch_bounds__(TX * TY) LBM_PHASE_OCC void k_phase(PhaseK k, const S* __restrict__ hc,
                                               S* __restrict__ hn, const S* __restrict__ zc,
                                               S* __restrict__ zn, S* __restrict__ phiu,
                                               double* __restrict__ mout) {
    constexpr bool RMASS = std::is_same<S, float>::value;
    __shared__ C sphi[TY + 2][TX + 2];
    const int nx = k.nx, ny = k.ny;
    const long long P = k.P;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int gx = (nx + TX - 1) / TX, gy = (ny + TY - 1) / TY;
    int tile;
    if (!xcd_tile(gx * gy * k.batch, tile)) return;  // whole workgroup, before any barrier
    const int b = tile / (gx * gy), r = tile - b * gx * gy;
    const int x0 = (r % gx) * TX, y0 = (r / gx) * TY;
    const long long base = (long long)b * ny * nx;
    const S* hlo_c = RMASS ? hc + 18 * P : nullptr;  // h_0 low part (plane 18)
    auto gxw = [&](int gx) { return ((gx % nx) + nx) % nx; };
    auto gyw = [&](int gy) {
        if (k.bcy) return gy < 0 ? 0 : (gy >= ny ? ny - 1 : gy);  // mirror ghost at walls
        return ((gy % ny) + ny) % ny;
    };
    // Every load of the tile is issued before the barrier: the node's own h, z
    // and (phi u) (kept in registers for the collision) and, for 140 threads,
    // the 10 values of one ring node; the barrier then waits for memory once.
    const int x = x0 + tx, y = y0 + ty;
    const bool valid = x < nx && y < ny;
    const long long n = base + (long long)gyw(y) * nx + gxw(x);  // == own node when valid
    C h[9], z[9], hlo = C(0), pu0 = C(0), pu1 = C(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = C(hc[i * P + n]);
    if (RMASS) hlo = C(hlo_c[n]);
    if (valid) {
#pragma unroll
        for (int i = 0; i < 9; ++i) z[i] = C(zc[i * P + n]);
        if constexpr (!MACROS) {
            pu0 = C(phiu[n]);
            pu1 = C(phiu[P + n]);
        }
    }
    int hx = -2, hy = -2;
    {
        const int t = ty * TX + tx;
        if (t < TX + 2) { hy = -1; hx = t - 1; }
        else if (t < 2 * (TX + 2)) { hy = TY; hx = t - (TX + 2) - 1; }
        else if (t < 2 * (TX + 2) + TY) { hx = -1; hy = t - 2 * (TX + 2); }
        else if (t < 2 * (TX + 2) + 2 * TY) { hx = TX; hy = t - 2 * (TX + 2) - TY; }
    }
    C ring = C(0);
    if (hx > -2) {
        const long long nn = base + (long long)gyw(y0 + hy) * nx + gxw(x0 + hx);
        ring = node_phi<S, C>(hc, hlo_c, P, nn);
    }
    // phi of the node, Eq. zero_moment_h (rest population with its low part)
    const C phi_own = (h[0] + hlo) + (((h[1] + h[3]) + (h[2] + h[4])) + ((h[5] + h[7]) + (h[6] + h[8])));
    sphi[ty + 1][tx + 1] = phi_own;
    if (hx > -2) sphi[hy + 1][hx + 1] = ring;
    __syncthreads();
    if (!valid) return;

    // ---- stencils, Eq. gradient and Eq. laplacian in lattice form:
    //      grad phi = 3 G / dx, lap phi = 6 L / dx^2
    const C phi = sphi[ty + 1][tx + 1];
    C Gx = C(0), Gy = C(0), Lp = C(0);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const C pn = sphi[ty + 1 + EY[i]][tx + 1 + EX[i]];
        Gx += wgt<C>(i) * C(EX[i]) * pn;
        Gy += wgt<C>(i) * C(EY[i]) * pn;
        Lp += wgt<C>(i) * (pn - phi);
    }
    const C drl = C(k.rho_l - k.rho_g);
    const C rho = C(k.rho_g) + phi * drl;  // linear in phi (Sec. 2.3)
    C nuh;
    if (k.visc_mode == 0) nuh = C(k.nuh_g) + phi * C(k.nuh_l - k.nuh_g);
    else nuh = (C(k.zh_g) + phi * C(k.zh_l - k.zh_g)) / rho;  // nu = zeta / rho (Sec. 4.4)
    const C wn = C(1) / (C(3) * nuh + C(0.5));                // dt / tau
    // chemical potential, Eq. chemical_potential; surface force F_s = mu grad phi
    const C mu = C(4) * C(k.beta) * phi * (phi - C(1)) * (phi - C(0.5)) - C(k.kap6) * Lp;
    const C fsx = mu * Gx * C(k.fs_scale) + C(k.Fbt[0]);
    const C fsy = mu * Gy * C(k.fs_scale) + C(k.Fbt[1]);
    // guarded interface normal (text after Eq. laplacian)
    const C gn2 = Gx * Gx + Gy * Gy;
    C nxv = C(0), nyv = C(0);
    if (gn2 > C(k.Geps) * C(k.Geps)) {
        const C ig = C(1) / sqrt(gn2);
        nxv = Gx * ig;
        nyv = Gy * ig;
    }
    // ---- pressure populations: velocity first (Eq. u_Liang), then pressure
    const C jx = (z[1] - z[3]) + ((z[5] - z[7]) + (z[8] - z[6]));
    const C jy = (z[2] - z[4]) + ((z[5] - z[7]) + (z[6] - z[8]));
    const C ir = C(1) / rho;
    const C ux = (jx + C(0.5) * fsx) * ir;
    const C uy = (jy + C(0.5) * fsy) * ir;
    const C uu = ux * ux + uy * uy;
    const C ug = ux * Gx + uy * Gy;
    const C zs = ((z[1] + z[3]) + (z[2] + z[4])) + ((z[5] + z[7]) + (z[6] + z[8]));
    // p / c_s^2, Eq. p_Liang: c_s^2/(1 - w_0) [sum_{i>0} z_i + dt/2 u.grad rho + rho s_0(u)]
    const C ph = C(1.8) * (zs + C(1.5) * drl * ug - C(1.5) * wgt<C>(0) * rho * uu);

    if constexpr (MACROS) {
        const long long Q = k.P;
        mout[0 * Q + n] = double(rho);
        mout[1 * Q + n] = double(ph) * k.cs2;
        mout[2 * Q + n] = double(ux) * k.c;
        mout[3 * Q + n] = double(uy) * k.c;
        mout[4 * Q + n] = 0.0;
        mout[5 * Q + n] = double(phi);
        mout[6 * Q + n] = double(mu);
        return;
    } else {
        // ---- interface populations (Eq. eq_lattice_boltzmann_interface,
        //      source_term_interface, heq_liang); d(phi u)/dt by explicit Euler
        const C pux = phi * ux, puy = phi * uy;
        const C dpx = pux - pu0, dpy = puy - pu1;
        st(phiu + n, S(pux));
        st(phiu + P + n, S(puy));
        const C wphi = C(k.w_phi);
        const C sfac = C(1) - C(0.5) * wphi;
        const C sharp = C(4) * phi * (C(1) - phi) * C(k.dxW);
        C hs[9];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const C eu = C(EX[i]) * ux + C(EY[i]) * uy;
            const C heq = phi * wgt<C>(i) * (C(1) + C(3) * eu);
            const C sh = sfac * wgt<C>(i) *
                         (C(3) * (C(EX[i]) * dpx + C(EY[i]) * dpy) +
                          sharp * (C(EX[i]) * nxv + C(EY[i]) * nyv));
            hs[i] = h[i] - wphi * (h[i] - heq) + sh;
        }
        S h0hi, h0lo = S(0);
        if constexpr (RMASS) {
            // rest population takes the node's exact balance: h0* = phi - sum_{i>0} h_i*
            // with the stored (rounded) h_i*, carried as a double-float
            float hi = float(h[0]), lo = float(hlo);
#pragma unroll
            for (int i = 1; i < 9; ++i) df_add(hi, lo, float(h[i]));
#pragma unroll
            for (int i = 1; i < 9; ++i) df_add(hi, lo, -float(hs[i]));
            h0hi = hi;
            h0lo = lo;
        } else {
            const C heq0 = phi * wgt<C>(0);
            h0hi = S(h[0] - wphi * (h[0] - heq0));
        }
        // ---- pressure collision in moment space.  The moments of z_i^eq
        //      (Eq. zeq_liang with Eq. s_i_Liang) and of dt F^z_i (Eq.
        //      forcing_term_pressure_evolution) under the integer matrix of
        //      Eq. M_matrix, in closed form:
        //        m^eq = (0, 2 p~ + 3 rho u^2, -3 (p~ + rho u^2), rho u_x, -rho u_x,
        //                rho u_y, -rho u_y, rho (u_x^2 - u_y^2), rho u_x u_y)
        //        m^F  = (3 D, 0, -3 D, F_x, -F_x, F_y, -F_y,
        //                2 drho (G_x u_x - G_y u_y), drho (G_x u_y + G_y u_x))
        //      with p~ = p / c_s^2, D = drho (u . G) and every velocity in units
        //      of c.  BGK is the same update with every rate equal to dt/tau.
        C m[9];
        moments9(z, m);
        {
            const C ruu = rho * uu, D = drl * ug;
            const C meq[9] = {C(0), C(2) * ph + C(3) * ruu, C(-3) * (ph + ruu), rho * ux, -rho * ux,
                              rho * uy, -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy};
            const C mf[9] = {C(3) * D, C(0), C(-3) * D, fsx, -fsx, fsy, -fsy,
                             C(2) * drl * (Gx * ux - Gy * uy), drl * (Gx * uy + Gy * ux)};
            const C wq = C(3) * (C(2) - wn) / (C(3) - wn);
            const C Lm[9] = {C(1), C(1), C(1), C(1), wq, C(1), k.qy_printed ? C(1) : wq, wn, wn};
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const C L = k.z_mrt ? Lm[q] : wn;
                m[q] += -L * (m[q] - meq[q]) + (C(1) - C(0.5) * L) * mf[q];
            }
        }
        C zst[9];
        inverse9(m, zst);
        // ---- streaming of h and z: x periodic; y periodic or halfway
        //      bounce-back walls
        st(hn + n, h0hi);
        if constexpr (RMASS) st(hn + 18 * P + n, h0lo);
        st(zn + n, S(zst[0]));
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int tyd = y + EY[i];
            if (k.bcy && (tyd < 0 || tyd >= ny)) {
                st(hn + OPP[i] * P + n, S(hs[i]));
                st(zn + OPP[i] * P + n, S(zst[i]));
            } else {
                const long long d = base + (long long)wrap(tyd, ny) * nx + wrap(x + EX[i], nx);
                st(hn + i * P + d, S(hs[i]));
                st(zn + i * P + d, S(zst[i]));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 1D thermal BGK, whole run in one block (n <= 1024): LDS streaming
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_d1(D1K k, double* __restrict__ g, int nsteps) {
    __shared__ double sg[3][1024];
    const int x = threadIdx.x;
    const int n = k.n, q = k.q;
    int ex[3];
    double w[3];
    if (q == 3) {
        ex[0] = 0; ex[1] = 1; ex[2] = -1;
        w[0] = 4.0 / 6; w[1] = 1.0 / 6; w[2] = 1.0 / 6;
    } else {
        ex[0] = 1; ex[1] = -1; ex[2] = 0;
        w[0] = 0.5; w[1] = 0.5; w[2] = 0.0;
    }
    double v[3] = {0, 0, 0};
    const bool act = x < n;
    if (act)
        for (int i = 0; i < q; ++i) v[i] = g[i * n + x];
    for (int s = 0; s < nsteps; ++s) {
        if (act) {
            double T = 0;
            for (int i = 0; i < q; ++i) T += v[i];
            T += 0.5 * k.qdt;
            for (int i = 0; i < q; ++i) {
                const double geq = w[i] * T * (1.0 + k.ufac * ex[i]);
                sg[i][x] = v[i] - k.w_tau * (v[i] - geq) + (1.0 - 0.5 * k.w_tau) * w[i] * k.qdt;
            }
        }
        __syncthreads();
        if (act) {
            int unknown = -1;
            double known = 0.0;
            for (int i = 0; i < q; ++i) {
                const int xs = x - ex[i];
                if (xs >= 0 && xs < n) {
                    v[i] = sg[i][xs];
                    known += v[i];
                } else {
                    unknown = i;
                }
            }
            if (unknown >= 0) {  // wet-node Dirichlet with the half source
                const double Tw = (x == 0) ? k.T0 : k.TL;
                v[unknown] = Tw - 0.5 * k.qdt - known;
            }
        }
        __syncthreads();
    }
    if (act)
        for (int i = 0; i < q; ++i) g[i * n + x] = v[i];
}

// ---------------------------------------------------------------------------
// initialisation from macroscopic fields (staging slots: 0 rho|p, 1 ux, 2 uy,
// 3 T, 4 phi; all FP64, velocities in m/s)
// ---------------------------------------------------------------------------
template <typename S>
__global__ void k_chan_init(ChanK k, const double* __restrict__ fld, S* __restrict__ f,
                            S* __restrict__ g) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    const long long P = k.P;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        const double rho = fld[n], ux = fld[P + n] / k.c, uy = fld[2 * P + n] / k.c;
        const double th = fld[3 * P + n] - k.T_ref;
        const double uu = ux * ux + uy * uy;
        for (int i = 0; i < 9; ++i) {
            const double eu = EX[i] * ux + EY[i] * uy;
            f[i * P + n] = S(wgt<double>(i) * ((rho - k.rho_ref) +
                                               rho * (3 * eu + 4.5 * eu * eu - 1.5 * uu)));
        }
        if (g)
            for (int i = 0; i < 5; ++i)
                g[i * P + n] = S(wgt5<double>(i) * th * (1 + 3 * (EX5[i] * ux + EY5[i] * uy)));
    }
}

template <typename S>
__global__ void k_phase_init(PhaseK k, const double* __restrict__ fld, S* __restrict__ h,
                             S* __restrict__ z, S* __restrict__ phiu) {
    constexpr bool RMASS = std::is_same<S, float>::value;
    const long long N = (long long)k.batch * k.nx * k.ny;
    const long long P = k.P;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        const double p = fld[n], ux = fld[P + n] / k.c, uy = fld[2 * P + n] / k.c;
        const double phi = fld[4 * P + n];
        const double rho = k.rho_g + phi * (k.rho_l - k.rho_g);
        const double ph = p / k.cs2, uu = ux * ux + uy * uy;
        double hsum = 0.0;
        for (int i = 1; i < 9; ++i) {
            const double eu = EX[i] * ux + EY[i] * uy;
            const S hv = S(phi * wgt<double>(i) * (1 + 3 * eu));
            h[i * P + n] = hv;
            hsum += double(hv);
        }
        const double h0 = phi - hsum;  // rest population closes the node's phi exactly
        const S hi = S(h0);
        h[n] = hi;
        if (RMASS) h[18 * P + n] = S(h0 - double(hi));
        for (int i = 0; i < 9; ++i) {
            const double eu = EX[i] * ux + EY[i] * uy;
            const double w = wgt<double>(i);
            z[i * P + n] = S(ph * (i == 0 ? w - 1 : w) + rho * w * (3 * eu + 4.5 * eu * eu - 1.5 * uu));
        }
        phiu[n] = S(phi * ux);
        phiu[P + n] = S(phi * uy);
    }
}

__global__ void k_d1_init(D1K k, const double* __restrict__ T, double* __restrict__ g) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= k.n) return;
    if (k.q == 3) {
        const double w[3] = {4.0 / 6, 1.0 / 6, 1.0 / 6};
        const int ex[3] = {0, 1, -1};
        for (int i = 0; i < 3; ++i) g[i * k.n + x] = w[i] * T[x] * (1 + k.ufac * ex[i]);
    } else {
        g[x] = 0.5 * T[x] * (1 + k.ufac);
        g[k.n + x] = 0.5 * T[x] * (1 - k.ufac);
    }
}

// ---------------------------------------------------------------------------
// FP64 macros of the stored state
// ---------------------------------------------------------------------------
template <typename S>
__global__ void k_chan_macros(ChanK k, const S* __restrict__ f, const S* __restrict__ g,
                              double* __restrict__ out) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    const long long P = k.P;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        double d[9], drho, rho, ux, uy;
        chan_flow_macros<double, S>(f, P, n, k.rho_ref, k.Ft[0], k.Ft[1], d, drho, rho, ux, uy);
        out[n] = rho;
        out[2 * P + n] = ux * k.c;
        out[3 * P + n] = uy * k.c;
        double T = k.T_ref;
        if (g) {
            double s = 0;
            for (int i = 0; i < 5; ++i) s += double(g[i * P + n]);
            T = k.T_ref + s + 0.5 * k.qdt;
        }
        out[4 * P + n] = T;
    }
}

__global__ void k_d1_macros(D1K k, const double* __restrict__ g, double* __restrict__ out,
                            long long P) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= k.n) return;
    double s = 0;
    for (int i = 0; i < k.q; ++i) s += g[i * k.n + x];
    out[4 * P + x] = s + 0.5 * k.qdt;
}

// ---------------------------------------------------------------------------
// deterministic FP64 reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NF>
__device__ void block_sums(double (&v)[NF], double* dst, int stride) {
    __shared__ double red[NF][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const double s = wave_sum(v[f]);
        if (lane == 0) red[f][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int f = 0; f < NF; ++f) dst[f * stride] = ((red[f][0] + red[f][1]) + red[f][2]) + red[f][3];
}

// pass 1: grid (kRedBlocks, batch), 256 threads; partial[(b*4 + f) * kRedBlocks + blk]
template <typename S>
__global__ __launch_bounds__(256) void k_reduce1(int lattice, ChanK ck, PhaseK pk, D1K dk,
                                                 const S* __restrict__ pops, int npop,
                                                 double* __restrict__ partial) {
    const int b = blockIdx.y;
    long long M, P;
    if (lattice == LBM_D2Q9_PHASE) { M = (long long)pk.nx * pk.ny; P = pk.P; }
    else if (lattice == LBM_D2Q9_D2Q5) { M = (long long)ck.nx * ck.ny; P = ck.P; }
    else { M = dk.n; P = dk.n; }
    const long long base = b * M;
    double v[4] = {0, 0, 0, 0};
    for (long long j = blockIdx.x * 256LL + threadIdx.x; j < M; j += 256LL * gridDim.x) {
        const long long n = base + j;
        double cnt = 0;
        for (int i = 0; i < npop; ++i) {
            const double a = double(pops[i * P + n]);
            if (!isfinite(a)) cnt += 1;
        }
        v[3] += cnt;
        if (lattice == LBM_D2Q9_PHASE) {
            double a = 0;
            for (int i = 0; i < 9; ++i) a += double(pops[i * P + n]);
            if (std::is_same<S, float>::value) a += double(pops[18 * P + n]);
            v[1] += a;
            v[0] += pk.rho_g + a * (pk.rho_l - pk.rho_g);
        } else if (lattice == LBM_D2Q9_D2Q5) {
            double a = 0;
            for (int i = 0; i < 9; ++i) a += double(pops[i * P + n]);
            v[0] += ck.rho_ref + a;
            if (ck.thermal) {
                double s = 0;
                for (int i = 0; i < 5; ++i) s += double(pops[(9 + i) * P + n]);
                v[2] += ck.T_ref + s + 0.5 * ck.qdt;
            }
        } else {
            double s = 0;
            for (int i = 0; i < dk.q; ++i) s += double(pops[i * dk.n + n]);
            v[2] += s + 0.5 * dk.qdt;
        }
    }
    block_sums<4>(v, partial + (long long)b * 4 * kRedBlocks + blockIdx.x, kRedBlocks);
}

// pass 2: one thread per (replica, field), fixed-order sum
__global__ void k_reduce2(const double* __restrict__ partial, double* __restrict__ out, int nb) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb * 4) return;
    const double* p = partial + (long long)t * kRedBlocks;
    double s = 0;
    for (int i = 0; i < kRedBlocks; ++i) s += p[i];
    out[t] = s;
}

// channel diagnostics of replica 0: one thread per column
template <typename S>
__global__ void k_nusselt(ChanK k, const S* __restrict__ f, const S* __restrict__ g,
                          const S* __restrict__ qw, double qsi, double Dh, double kc, double dx,
                          double* __restrict__ Tb, double* __restrict__ Tw,
                          double* __restrict__ Nu) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= k.nx) return;
    const long long P = k.P;
    double su = 0, suT = 0, T0 = 0, T1 = 0;
    for (int y = 0; y < k.ny; ++y) {
        const long long n = (long long)y * k.nx + x;
        double d[9], drho, rho, ux, uy;
        chan_flow_macros<double, S>(f, P, n, k.rho_ref, k.Ft[0], k.Ft[1], d, drho, rho, ux, uy);
        double s = 0;
        for (int i = 0; i < 5; ++i) s += double(g[i * P + n]);
        const double T = k.T_ref + s + 0.5 * k.qdt;
        su += ux;
        suT += ux * T;
        if (y == 0) T0 = T;
        if (y == k.ny - 1) T1 = T;
    }
    const double q = double(qw[x]) * qsi;  // W/m^2 including the time modulation
    const double tb = suT / su;
    const double tw = 0.5 * (T0 + T1) + q * dx / (2.0 * kc);
    Tb[x] = tb;
    Tw[x] = tw;
    Nu[x] = q * Dh / (kc * (tw - tb));
}

__global__ void k_nusselt_mean(const double* __restrict__ Nu, const double* __restrict__ Tb,
                               int nx, int x_dev, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0;
    for (int x = x_dev; x < nx; ++x) s += Nu[x];
    out[0] = s / double(nx - x_dev);
    out[1] = Tb[nx - 1];
}

inline unsigned grid1(long long N, int bs) {
    long long g = (N + bs - 1) / bs;
    if (g > 65535LL * 16) g = 65535LL * 16;
    return unsigned(g < 1 ? 1 : g);
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
template <typename S>
hipError_t launch_chan_step(const ChanK& k, const S* fc, S* fn, const S* gc, S* gn, const S* qw,
                            const S* uin, const S* tin, double mod, hipStream_t s) {
    const long long tiles = (long long)((k.nx + 63) / 64) * ((k.ny + 3) / 4) * k.batch;
    dim3 blk(64, 4), grd(unsigned((tiles + kXCD - 1) / kXCD * kXCD));
    hipLaunchKernelGGL(k_chan_step<S>, grd, blk, 0, s, k, fc, fn, gc, gn, qw, uin, tin, S(mod));
    return hipGetLastError();
}

template <typename S>
hipError_t launch_phase_step(const PhaseK& k, const S* hc, S* hn, const S* zc, S* zn, S* phiu,
                             hipStream_t s) {
    const long long tiles = (long long)((k.nx + TX - 1) / TX) * ((k.ny + TY - 1) / TY) * k.batch;
    dim3 blk(TX, TY), grd(unsigned((tiles + kXCD - 1) / kXCD * kXCD));
    const unsigned lds = std::is_same<S, float>::value ? kPhaseLdsReserve : 0u;
    hipLaunchKernelGGL((k_phase<S, S, false>), grd, blk, lds, s, k, hc, hn, zc, zn, phiu,
                       (double*)nullptr);
    return hipGetLastError();
}

hipError_t launch_d1(const D1K& k, double* g, int nsteps, hipStream_t s) {
    hipLaunchKernelGGL(k_d1, dim3(1), dim3(1024), 0, s, k, g, nsteps);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_chan_init(const ChanK& k, const double* fields, S* f, S* g, hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    hipLaunchKernelGGL(k_chan_init<S>, dim3(grid1(N, 256)), dim3(256), 0, s, k, fields, f, g);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_phase_init(const PhaseK& k, const double* fields, S* h, S* z, S* phiu,
                             hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    hipLaunchKernelGGL(k_phase_init<S>, dim3(grid1(N, 256)), dim3(256), 0, s, k, fields, h, z,
                       phiu);
    return hipGetLastError();
}

hipError_t launch_d1_init(const D1K& k, const double* T, double* g, hipStream_t s) {
    hipLaunchKernelGGL(k_d1_init, dim3((k.n + 255) / 256), dim3(256), 0, s, k, T, g);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_chan_macros(const ChanK& k, const S* f, const S* g, double* out,
                              hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    hipLaunchKernelGGL(k_chan_macros<S>, dim3(grid1(N, 256)), dim3(256), 0, s, k, f, g, out);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_phase_macros(const PhaseK& k, const S* h, const S* z, double* out,
                               hipStream_t s) {
    const long long tiles = (long long)((k.nx + TX - 1) / TX) * ((k.ny + TY - 1) / TY) * k.batch;
    dim3 blk(TX, TY), grd(unsigned((tiles + kXCD - 1) / kXCD * kXCD));
    hipLaunchKernelGGL((k_phase<S, double, true>), grd, blk, 0, s, k, h, (S*)nullptr, z,
                       (S*)nullptr, (S*)nullptr, out);
    return hipGetLastError();
}

hipError_t launch_d1_macros(const D1K& k, const double* g, double* out, long long P,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_d1_macros, dim3((k.n + 255) / 256), dim3(256), 0, s, k, g, out, P);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_reduce(int lattice, const ChanK& ck, const PhaseK& pk, const D1K& dk,
                         const S* pops, int npop, double* partial, double* out, hipStream_t s) {
    int batch = lattice == LBM_D2Q9_PHASE ? pk.batch : (lattice == LBM_D2Q9_D2Q5 ? ck.batch : 1);
    hipLaunchKernelGGL(k_reduce1<S>, dim3(kRedBlocks, batch), dim3(256), 0, s, lattice, ck, pk,
                       dk, pops, npop, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce2, dim3((batch * 4 + 63) / 64), dim3(64), 0, s, partial, out,
                       batch);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_nusselt(const ChanK& k, const S* f, const S* g, const S* qw, double qsi,
                          double Dh, double kc, double dx, int x_dev, double* Tb, double* Tw,
                          double* Nu, double* small, hipStream_t s) {
    hipLaunchKernelGGL(k_nusselt<S>, dim3((k.nx + 255) / 256), dim3(256), 0, s, k, f, g, qw, qsi,
                       Dh, kc, dx, Tb, Tw, Nu);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nusselt_mean, dim3(1), dim3(64), 0, s, Nu, Tb, k.nx, x_dev, small);
    return hipGetLastError();
}

#define LBM_INST(S)                                                                              \
    template hipError_t launch_chan_step<S>(const ChanK&, const S*, S*, const S*, S*, const S*, \
                                            const S*, const S*, double, hipStream_t);             \
    template hipError_t launch_phase_step<S>(const PhaseK&, const S*, S*, const S*, S*, S*,      \
                                             hipStream_t);                                        \
    template hipError_t launch_chan_init<S>(const ChanK&, const double*, S*, S*, hipStream_t);   \
    template hipError_t launch_phase_init<S>(const PhaseK&, const double*, S*, S*, S*,           \
                                             hipStream_t);                                        \
    template hipError_t launch_chan_macros<S>(const ChanK&, const S*, const S*, double*,         \
                                              hipStream_t);                                       \
    template hipError_t launch_phase_macros<S>(const PhaseK&, const S*, const S*, double*,       \
                                               hipStream_t);                                      \
    template hipError_t launch_reduce<S>(int, const ChanK&, const PhaseK&, const D1K&, const S*, \
                                         int, double*, double*, hipStream_t);                     \
    template hipError_t launch_nusselt<S>(const ChanK&, const S*, const S*, const S*, double,    \
                                          double, double, double, int, double*, double*, double*, \
                                          double*, hipStream_t);
LBM_INST(float)
LBM_INST(double)

}  // namespace lbm

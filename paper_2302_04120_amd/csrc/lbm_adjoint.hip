// Discrete adjoint of the D2Q9 (BGK/MRT) + D2Q5 heated-channel step.
//
// One forward step maps the pre-collision state s(n) = (f, g) to s(n+1) by
// macros -> collision -> push-streaming with the boundary rules.  The reverse
// step applies the transpose of that map's Jacobian to the adjoint state
// lambda(n+1) and returns lambda(n).  It is written in gather form: the node
// reads the adjoint values at the slots its own post-collision populations were
// written to (the transpose of the push, including each boundary rule), applies
// the transposed collision of the thermal and then the momentum populations,
// and writes lambda(n) at its own slots only, so no two threads write the same
// value.  The moment-space relaxation operators M^-1 diag(L) M are symmetric
// (the rows of M are orthogonal), so their transposes are the same transforms.
//
// Parameter gradients accumulate in FP64 with one owner per accumulator: the
// wall-flux gradient per column and wall (the wall-node thread), the
// relaxation-time gradients per tile (thread 0 of the tile's workgroup, the
// tile-to-workgroup map being fixed), then summed in a fixed order.
#include "lbm_device.h"

#include <cmath>

namespace lbm {
namespace {

constexpr double kD9[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};  // squared row norms of M
constexpr double kD5[5] = {5, 2, 2, 20, 4};

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename S>
__global__ __launch_bounds__(256) void k_adj_step(ChanK k, AdjK a, const S* __restrict__ st,
                                                  const S* __restrict__ ln,
                                                  S* __restrict__ l, S mod,
                                                  double* __restrict__ dq_bot,
                                                  double* __restrict__ dq_top,
                                                  double* __restrict__ dtau_acc) {
    using C = S;
    __shared__ double red[2][4];
    const int nx = k.nx, ny = k.ny;
    const int gx = (nx + 63) / 64, gy = (ny + 3) / 4;
    int tile;
    if (!xcd_tile(gx * gy, tile)) return;  // whole workgroup, before the barrier
    const int x = (tile % gx) * 64 + threadIdx.x;
    const int y = (tile / gx) * 4 + threadIdx.y;
    const bool active = x < nx && y < ny;
    const int npl = k.npl;  // node blocks: f 0-8, g 9-13
    double dtn = 0.0, dtt = 0.0;
    if (active) {
        const long long n = (long long)y * nx + x;
        const C rho_ref = C(k.rho_ref), ftx = C(k.Ft[0]), fty = C(k.Ft[1]);
        C d[9], drho, rho, ux, uy;
        chan_flow_macros<C, S>(st, npl, n, rho_ref, ftx, fty, d, drho, rho, ux, uy);
        C e[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) e[i] = C(st[bidx(npl, 9 + i, n)]);
        const C qdt = C(k.qdt);
        const C th = (e[0] + (e[1] + e[3]) + (e[2] + e[4])) + C(0.5) * qdt;

        // ---- transpose of streaming and the momentum boundary rules
        C ubx = C(0), uby = C(0);  // adjoint of the lattice velocity u / c
        C uwx = C(0), uwy = C(0);
        if (k.bcx && x == nx - 1) {
            C d2[9], dr2, r2, ux2, uy2;
            chan_flow_macros<C, S>(st, npl, n - 1, rho_ref, ftx, fty, d2, dr2, r2, ux2, uy2);
            uwx = C(1.5) * ux - C(0.5) * ux2;
            uwy = C(1.5) * uy - C(0.5) * uy2;
        }
        C ls[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int tx = x + EX[i], ty = y + EY[i];
            const bool outy = k.bcy && (ty < 0 || ty >= ny);
            const bool outx = k.bcx && (tx < 0 || tx >= nx);
            if (!outy && !outx) {
                tx = wrap(tx, nx);
                ty = wrap(ty, ny);
                ls[i] = C(ln[bidx(npl, i, (long long)ty * nx + tx)]);
            } else if (outy || tx < 0) {
                ls[i] = C(ln[bidx(npl, OPP[i], n)]);  // bounce-back (wall, moving inlet)
            } else {
                // anti-bounce-back outlet: -f_i* + 2 w rho_ref [4.5 (e.u_w)^2 - 1.5 u_w^2]
                const C lam = C(ln[bidx(npl, OPP[i], n)]);
                ls[i] = -lam;
                const C eu = C(EX[i]) * uwx + C(EY[i]) * uwy;
                const C k2 = C(2) * wgt<C>(i) * rho_ref;
                // u_w = 1.5 u(x_b) - 0.5 u(x_b - 1): this node's share
                ubx += C(1.5) * lam * k2 * (C(9) * eu * C(EX[i]) - C(3) * uwx);
                uby += C(1.5) * lam * k2 * (C(9) * eu * C(EY[i]) - C(3) * uwy);
            }
        }
        if (k.bcx && nx >= 2 && x == nx - 2) {
            // the outlet node to the right depends on this node's velocity
            C d2[9], dr2, r2, ux2, uy2;
            chan_flow_macros<C, S>(st, npl, n + 1, rho_ref, ftx, fty, d2, dr2, r2, ux2, uy2);
            const C vx = C(1.5) * ux2 - C(0.5) * ux, vy = C(1.5) * uy2 - C(0.5) * uy;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (EX[i] != 1) continue;
                const int ty = y + EY[i];
                if (k.bcy && (ty < 0 || ty >= ny)) continue;  // wall rule at the corner
                const C lam = C(ln[bidx(npl, OPP[i], n + 1)]);
                const C eu = C(EX[i]) * vx + C(EY[i]) * vy;
                const C k2 = C(2) * wgt<C>(i) * rho_ref;
                ubx += C(-0.5) * lam * k2 * (C(9) * eu * C(EX[i]) - C(3) * vx);
                uby += C(-0.5) * lam * k2 * (C(9) * eu * C(EY[i]) - C(3) * vy);
            }
        }
        // ---- transpose of streaming and the thermal boundary rules
        C lsg[5];
        double dqb = 0.0, dqt = 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            int tx = x + EX5[i], ty = y + EY5[i];
            const bool outy = k.bcy && (ty < 0 || ty >= ny);
            const bool outx = k.bcx && (tx < 0 || tx >= nx);
            if (!outy && !outx) {
                tx = wrap(tx, nx);
                ty = wrap(ty, ny);
                lsg[i] = C(ln[bidx(npl, 9 + i, (long long)ty * nx + tx)]);
            } else if (outy) {
                // flux wall: + lambda (dt/dx) q'' / rho c_p
                const C lam = C(ln[bidx(npl, 9 + OPP5[i], n)]);
                lsg[i] = lam;
                const double gq = double(lam) * a.qgrad * double(mod);
                if (ty < 0) dqb += gq;
                else dqt += gq;
            } else if (tx < 0) {
                lsg[i] = -C(ln[bidx(npl, 9 + OPP5[i], n)]);  // anti-bounce-back inlet
            } else {
                lsg[i] = C(0);  // dropped at the extrapolation outlet
            }
        }
        if (k.bcx && x == nx - 1) lsg[3] += C(ln[bidx(npl, 9 + 3, n)]);  // outlet slot took g_3*
        // ---- transpose of the thermal collision g* = g - A_T (g - g_eq(T, u)) + B_T S
        {
            C mL[5], mN[5], neq[5], tmp[5], ag[5];
            moments5(lsg, mL);
#pragma unroll
            for (int i = 0; i < 5; ++i)
                neq[i] = e[i] - wgt5<C>(i) * th * (C(1) + C(3) * (C(EX5[i]) * ux + C(EY5[i]) * uy));
            moments5(neq, mN);
            const double ms[5] = {double(qdt), 0.0, 0.0, -2.0 / 3.0 * double(qdt), 0.0};
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                tmp[q] = C(k.Lt[q]) * mL[q];
                dtt += double(mL[q]) / kD5[q] * (-a.dLt[q] * double(mN[q]) - 0.5 * a.dLt[q] * ms[q]);
            }
            inverse5(tmp, ag);  // A_T lambda* (A_T is symmetric)
            C tb = C(0);
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const C eu = C(EX5[i]) * ux + C(EY5[i]) * uy;
                tb += ag[i] * wgt5<C>(i) * (C(1) + C(3) * eu);
                ubx += ag[i] * wgt5<C>(i) * th * C(3) * C(EX5[i]);
                uby += ag[i] * wgt5<C>(i) * th * C(3) * C(EY5[i]);
            }
#pragma unroll
            for (int i = 0; i < 5; ++i) l[bidx(npl, 9 + i, n)] = S(lsg[i] - ag[i] + tb);
        }
        // ---- transpose of the momentum collision f* = f - A (f - f_eq(rho, u)) + B F(u)
        {
            const C uu = ux * ux + uy * uy;
            C neq[9], fh[9], av[9], bv[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const C eu = C(EX[i]) * ux + C(EY[i]) * uy;
                neq[i] = d[i] - wgt<C>(i) * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu));
                fh[i] = wgt<C>(i) * ((C(3) * (C(EX[i]) - ux) + C(9) * eu * C(EX[i])) * ftx +
                                     (C(3) * (C(EY[i]) - uy) + C(9) * eu * C(EY[i])) * fty);
            }
            if (k.flow_mrt) {
                C mL[9], mN[9], mF[9], t1[9], t2[9];
                moments9(ls, mL);
                moments9(neq, mN);
                moments9(fh, mF);
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const C L = C(k.Lf[q]);
                    t1[q] = L * mL[q];
                    t2[q] = (C(1) - C(0.5) * L) * mL[q];
                    dtn += double(mL[q]) / kD9[q] *
                           (-a.dLf[q] * double(mN[q]) - 0.5 * a.dLf[q] * double(mF[q]));
                }
                inverse9(t1, av);
                inverse9(t2, bv);
            } else {
                const C L = C(k.Lf[7]);
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    av[i] = L * ls[i];
                    bv[i] = (C(1) - C(0.5) * L) * ls[i];
                    dtn += double(ls[i]) * (-a.dLf[7] * double(neq[i]) - 0.5 * a.dLf[7] * double(fh[i]));
                }
            }
            C rb = C(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const C eu = C(EX[i]) * ux + C(EY[i]) * uy;
                const C w = wgt<C>(i);
                rb += av[i] * w * (C(1) + C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu);
                ubx += av[i] * w * rho * (C(3) * C(EX[i]) + C(9) * eu * C(EX[i]) - C(3) * ux);
                uby += av[i] * w * rho * (C(3) * C(EY[i]) + C(9) * eu * C(EY[i]) - C(3) * uy);
                const C eF = C(EX[i]) * ftx + C(EY[i]) * fty;
                ubx += bv[i] * w * (C(-3) * ftx + C(9) * C(EX[i]) * eF);
                uby += bv[i] * w * (C(-3) * fty + C(9) * C(EY[i]) * eF);
            }
            const C ir = C(1) / rho;
#pragma unroll
            for (int i = 0; i < 9; ++i)
                l[bidx(npl, i, n)] = S(ls[i] - av[i] + rb +
                                  ((C(EX[i]) - ux) * ubx + (C(EY[i]) - uy) * uby) * ir);
        }
        if (k.bcy && y == 0) dq_bot[x] += dqb;
        if (k.bcy && y == ny - 1) dq_top[x] += dqt;
    }
    // ---- per-tile FP64 sums of the relaxation-time gradients
    const int lane = (threadIdx.y * 64 + threadIdx.x) & 63, wv = threadIdx.y;
    const double sn = wave_sum64(dtn), st_ = wave_sum64(dtt);
    if (lane == 0) {
        red[0][wv] = sn;
        red[1][wv] = st_;
    }
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        dtau_acc[2 * tile] += ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        dtau_acc[2 * tile + 1] += ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

// Objective J = w_tout T_out + w_nu mean_{x >= x_dev} Nu(x) at the final state
// (definitions as in lbm_nusselt); one thread per column.
template <typename S>
__global__ void k_adj_seed(ChanK k, const S* __restrict__ st, const S* __restrict__ qw, double qsi, double mod, double Dh, double kc,
                           double dx, double rho_cp, double cs2, int x_dev, double w_tout,
                           double w_nu, S* __restrict__ l,
                           double* __restrict__ dq_direct, double* __restrict__ dtauT_direct) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = k.nx, ny = k.ny;
    if (x >= nx) return;
    const int npl = k.npl;  // node blocks: f 0-8, g 9-13
    double su = 0, suT = 0, T0 = 0, T1 = 0;
    for (int y = 0; y < ny; ++y) {
        const long long n = (long long)y * nx + x;
        double d[9], drho, rho, ux, uy;
        chan_flow_macros<double, S>(st, npl, n, k.rho_ref, k.Ft[0], k.Ft[1], d, drho, rho, ux,
                                    uy);
        double s = 0;
        for (int i = 0; i < 5; ++i) s += double(st[bidx(npl, 9 + i, n)]);
        const double T = k.T_ref + s + 0.5 * k.qdt;
        su += ux * k.c;
        suT += ux * k.c * T;
        if (y == 0) T0 = T;
        if (y == ny - 1) T1 = T;
    }
    const double q = double(qw[x]) * qsi;
    const double tb = suT / su;
    const double dT = 0.5 * (T0 + T1) + q * dx / (2.0 * kc) - tb;
    double bTb = (x == nx - 1) ? w_tout : 0.0, bTw = 0.0, dqd = 0.0, dtd = 0.0;
    if (x >= x_dev) {
        const double nu_x = q * Dh / (kc * dT);
        const double bNu = w_nu / double(nx - x_dev);
        const double bdT = -bNu * nu_x / dT;
        bTw += bdT;
        bTb -= bdT;
        dqd = bNu * mod * Dh / (kc * dT) + bdT * mod * dx / (2.0 * kc);
        dtd = bNu * (-nu_x / kc + (nu_x / dT) * q * dx / (2.0 * kc * kc)) * rho_cp * cs2;
    }
    dq_direct[x] = dqd;
    dtauT_direct[x] = dtd;
    for (int y = 0; y < ny; ++y) {
        const long long n = (long long)y * nx + x;
        double d[9], drho, rho, ux, uy;
        chan_flow_macros<double, S>(st, npl, n, k.rho_ref, k.Ft[0], k.Ft[1], d, drho, rho, ux,
                                    uy);
        double s = 0;
        for (int i = 0; i < 5; ++i) s += double(st[bidx(npl, 9 + i, n)]);
        const double T = k.T_ref + s + 0.5 * k.qdt;
        double Tbar = bTb * ux * k.c / su;
        if (y == 0) Tbar += 0.5 * bTw;
        if (y == ny - 1) Tbar += 0.5 * bTw;
        const double Ubar = bTb * (T - tb) / su * k.c;  // adjoint of u_x / c
        for (int i = 0; i < 5; ++i) l[bidx(npl, 9 + i, n)] = S(Tbar);
        for (int i = 0; i < 9; ++i) l[bidx(npl, i, n)] = S(Ubar * (EX[i] - ux) / rho);
    }
}

__global__ void k_adj_final(int nx, int ntiles, double scale, const double* __restrict__ dq_bot,
                            const double* __restrict__ dq_top,
                            const double* __restrict__ dq_direct,
                            const double* __restrict__ dtauT_direct,
                            const double* __restrict__ dtau_acc, double* __restrict__ grad_flux,
                            double* __restrict__ grad_tau) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nx) grad_flux[t] = scale * ((dq_bot[t] + dq_top[t]) + dq_direct[t]);
    if (t == 0) {
        double sn = 0, st = 0;
        for (int i = 0; i < ntiles; ++i) {
            sn += dtau_acc[2 * i];
            st += dtau_acc[2 * i + 1];
        }
        for (int x = 0; x < nx; ++x) st += dtauT_direct[x];
        grad_tau[0] = scale * sn;
        grad_tau[1] = scale * st;
    }
}

}  // namespace

int chan_tiles(const ChanK& k) { return ((k.nx + 63) / 64) * ((k.ny + 3) / 4); }

template <typename S>
hipError_t launch_adj_seed(const ChanK& k, const S* st, const S* qw, double qsi, double mod,
                           double Dh, double kc, double dx, double rho_cp, double cs2, int x_dev,
                           double w_tout, double w_nu, S* l, double* dq_direct,
                           double* dtauT_direct, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_seed<S>, dim3((k.nx + 63) / 64), dim3(64), 0, s, k, st, qw, qsi, mod,
                       Dh, kc, dx, rho_cp, cs2, x_dev, w_tout, w_nu, l, dq_direct, dtauT_direct);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_adj_step(const ChanK& k, const AdjK& a, const S* st, const S* ln, S* l,
                           double mod, double* dq_bot, double* dq_top, double* dtau_acc,
                           hipStream_t s) {
    const int tiles = chan_tiles(k);
    dim3 blk(64, 4), grd(unsigned((tiles + kXCD - 1) / kXCD * kXCD));
    hipLaunchKernelGGL(k_adj_step<S>, grd, blk, 0, s, k, a, st, ln, l, S(mod), dq_bot, dq_top,
                       dtau_acc);
    return hipGetLastError();
}

hipError_t launch_adj_final(int nx, int ntiles, double scale, const double* dq_bot,
                            const double* dq_top, const double* dq_direct,
                            const double* dtauT_direct, const double* dtau_acc, double* grad_flux,
                            double* grad_tau, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_final, dim3((nx + 255) / 256), dim3(256), 0, s, nx, ntiles, scale,
                       dq_bot, dq_top, dq_direct, dtauT_direct, dtau_acc, grad_flux, grad_tau);
    return hipGetLastError();
}

#define LBM_ADJ_INST(S)                                                                          \
    template hipError_t launch_adj_seed<S>(const ChanK&, const S*, const S*, double, double,     \
                                           double, double, double, double, double, int, double,   \
                                           double, S*, double*, double*, hipStream_t);            \
    template hipError_t launch_adj_step<S>(const ChanK&, const AdjK&, const S*, const S*, S*,    \
                                           double, double*, double*, double*, hipStream_t);
LBM_ADJ_INST(float)
LBM_ADJ_INST(double)

}  // namespace lbm

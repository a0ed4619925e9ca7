// HIP kernels of the dimensional LBM hot path for gfx950 (CDNA4, wave64).
//
// Data layout: node n = (b * ny + y) * nx + x (x fastest); the 2D states in
// node blocks (value i of node n at bidx(npl, i, n): the npl values of 64
// consecutive nodes together), the 1D lattices and the FP64 staging fields in
// planes of stride P.
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

// Thermal lattice of the channel: D2Q5 (QT = 5) or D2Q9 (QT = 9, the set of
// Sec. 3 and App. D).
template <int QT> __device__ __forceinline__ int tex(int i) { return QT == 9 ? EX[i] : EX5[i]; }
template <int QT> __device__ __forceinline__ int tey(int i) { return QT == 9 ? EY[i] : EY5[i]; }
template <int QT> __device__ __forceinline__ int topp(int i) { return QT == 9 ? OPP[i] : OPP5[i]; }
template <int QT> __device__ __forceinline__ int tmir(int i) { return QT == 9 ? MIRY[i] : MIRY5[i]; }
template <int QT, typename C> __device__ __forceinline__ C twt(int i) {
    return QT == 9 ? wgt<C>(i) : wgt5<C>(i);
}

// ---- per-node pieces of the channel step, shared by the one- and two-step
//      kernels so that both round identically
// T - T_ref of a node from its (deviation) thermal populations, with the half
// source (Eq. zero_moment_g)
template <int QT, typename C>
__device__ __forceinline__ C chan_th(const C (&e)[QT], C qdt) {
    if constexpr (QT == 9)
        return ((e[0] + (e[1] + e[3]) + (e[2] + e[4])) + ((e[5] + e[7]) + (e[6] + e[8]))) +
               C(0.5) * qdt;
    else
        return (e[0] + (e[1] + e[3]) + (e[2] + e[4])) + C(0.5) * qdt;
}

// Both collisions of a node: ds from the deviations d (Eq. colisao_MRT or Eq.
// eq_lattice_boltzmann_BGK with Guo forcing; a frozen flow keeps d), es from
// the thermal populations e (Sec. 2.2 and Sec. 3, advective part built on
// T - T_ref, in moment space with the rates Lt).
template <typename C, int QT>
__device__ __forceinline__ void chan_collide(const ChanK& k, const C (&d)[9], C drho, C rho, C ux,
                                             C uy, C ftx, C fty, const C (&e)[QT], C th, C qdt,
                                             C (&ds)[9], C (&es)[QT]) {
    if (k.flow) {
        const C uu = ux * ux + uy * uy;
        if (k.flow_mrt) {
            // Moment space: the non-equilibrium moments are M d minus the
            // moments of the deviation equilibrium (Eq. feq_geral less
            // w_i rho_ref) in closed form, (drho, -2 drho + 3 rho |u|^2,
            // drho - 3 rho |u|^2, rho u_x, -rho u_x, rho u_y, -rho u_y,
            // rho (u_x^2 - u_y^2), rho u_x u_y); the Guo term of Eq.
            // forcing_term has the moments (0, 6 u.F, -6 u.F, F_x, -F_x, F_y,
            // -F_y, 2 (u_x F_x - u_y F_y), u_x F_y + u_y F_x).
            C md[9], dm[9], dv[9];
            moments9(d, md);
            const C ru2 = rho * uu, rux = rho * ux, ruy = rho * uy;
            const C mn[9] = {md[0] - drho,
                             md[1] - (C(-2) * drho + C(3) * ru2),
                             md[2] - (drho - C(3) * ru2),
                             md[3] - rux,
                             md[4] + rux,
                             md[5] - ruy,
                             md[6] + ruy,
                             md[7] - (rux * ux - ruy * uy),
                             md[8] - rux * uy};
            const C uf = ux * ftx + uy * fty;
            const C mf[9] = {C(0),  C(6) * uf, C(-6) * uf, ftx, -ftx, fty, -fty,
                             C(2) * (ux * ftx - uy * fty), ux * fty + uy * ftx};
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const C L = C(k.Lf[q]);
                dm[q] = -L * mn[q] + (C(1) - C(0.5) * L) * mf[q];
            }
            inverse9(dm, dv);
#pragma unroll
            for (int i = 0; i < 9; ++i) ds[i] = d[i] + dv[i];
        } else {
            C neq[9], fh[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const C eu = C(EX[i]) * ux + C(EY[i]) * uy;
                // deviation of Eq. feq_geral from w_i rho_ref
                const C feq =
                    wgt<C>(i) * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu));
                neq[i] = d[i] - feq;
                // dt * Guo term of Eq. forcing_term (without its prefactor)
                fh[i] = wgt<C>(i) * ((C(3) * (C(EX[i]) - ux) + C(9) * eu * C(EX[i])) * ftx +
                                     (C(3) * (C(EY[i]) - uy) + C(9) * eu * C(EY[i])) * fty);
            }
            const C L = C(k.Lf[7]);
#pragma unroll
            for (int i = 0; i < 9; ++i) ds[i] = d[i] - L * neq[i] + (C(1) - C(0.5) * L) * fh[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) ds[i] = d[i];
    }
    if (k.thermal) {
        C m[QT], dm[QT], dv[QT];
        if constexpr (QT == 9) {
            C neq[9];
#pragma unroll
            for (int i = 0; i < 9; ++i)
                neq[i] = e[i] - twt<QT, C>(i) * th *
                                    (C(1) + C(3) * (C(tex<QT>(i)) * ux + C(tey<QT>(i)) * uy));
            moments9(neq, m);
            // moments of the source w_i qdot dt: qdt (1, -2, 1, 0, ...)
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const C L = C(k.Lt[q]);
                const C ms = q == 0 ? qdt : (q == 1 ? C(-2) * qdt : (q == 2 ? qdt : C(0)));
                dm[q] = -L * m[q] + (C(1) - C(0.5) * L) * ms;
            }
            inverse9(dm, dv);
        } else {
            // moments of e less those of the equilibrium w_i th (1 + 3 c_i.u):
            // (th, th u_x, th u_y, -2/3 th, 0)
            C me[5];
            moments5(e, me);
            m[0] = me[0] - th;
            m[1] = me[1] - th * ux;
            m[2] = me[2] - th * uy;
            m[3] = me[3] - C(-2) / C(3) * th;
            m[4] = me[4];
            // moments of the source w_i qdot dt: qdt (1, 0, 0, -2/3, 0)
            const C ms[5] = {qdt, C(0), C(0), C(-2) / C(3) * qdt, C(0)};
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const C L = C(k.Lt[q]);
                dm[q] = -L * m[q] + (C(1) - C(0.5) * L) * ms[q];
            }
            inverse5(dm, dv);
        }
#pragma unroll
        for (int i = 0; i < QT; ++i) es[i] = e[i] + dv[i];
    }
}

// Values a boundary rule puts into the node's opposite slot OPP[i] for a
// population i that leaves the domain:
// moving-wall bounce-back with the inlet profile u_in (Eq. BB_vel)
template <typename C>
__device__ __forceinline__ C chan_inlet_f(int i, C dsi, C rho_ref, C uin) {
    return dsi - C(6) * wgt<C>(i) * rho_ref * (C(EX[i]) * uin);
}
// anti-bounce-back pressure outlet with the wall velocity u_w (Eq.
// anti_BB_vel, rho_w = rho_ref)
template <typename C>
__device__ __forceinline__ C chan_outlet_f(int i, C dsi, C rho_ref, C uwx, C uwy) {
    const C eu = C(EX[i]) * uwx + C(EY[i]) * uwy;
    return -dsi + C(2) * wgt<C>(i) * rho_ref * (C(4.5) * eu * eu - C(1.5) * (uwx * uwx + uwy * uwy));
}
// prescribed wall flux q (scaled, times the time modulation mod), Eq. BB_T
// with lambda_i = 6 w_i (1 on D2Q5), into slot topp(i)
template <int QT, typename C>
__device__ __forceinline__ C chan_flux_g(int i, C esi, C q, C mod) {
    const C lam = QT == 9 ? C(6) * wgt<C>(i) : C(1);
    return esi + lam * q * mod;
}
// anti-bounce-back fixed temperature tw (deviation form, Eq. anti_BB_T), into
// slot topp(i)
template <int QT, typename C>
__device__ __forceinline__ C chan_antibb_g(int i, C esi, C tw) {
    return -esi + C(2) * twt<QT, C>(i) * tw;
}

// One step of the channel model: D2Q9 flow (BGK or dimensional MRT, Guo
// forcing, optional Boussinesq force) + D2Q5 or D2Q9 temperature.  Tiles of
// 64 nodes of one row (one wave each).  y: periodic (bcy 0), halfway walls
// (1), or a wall at y- and the symmetry plane of Eq. simetria at y+ (2).  x:
// periodic (bcx 0), velocity inlet + pressure outlet (1), fixed-temperature
// walls (2).
template <typename S, int QT>
__global__ __launch_bounds__(64) void k_chan_step(ChanK k, const S* __restrict__ A,
                                                        S* __restrict__ B, const S* __restrict__ qw,
                                                        const S* __restrict__ uin,
                                                        const S* __restrict__ tin, S mod) {
    using C = S;
    const int nx = k.nx, ny = k.ny;
    const int gx = (nx + 63) / 64;
    int tile;
    if (!xcd_tile(gx * ny * k.batch, tile)) return;
    const int b = tile / (gx * ny), r = tile - b * gx * ny;
    const int x = (r % gx) * 64 + threadIdx.x;
    const int y = r / gx;
    if (x >= nx) return;
    const int npl = k.npl;  // node blocks: f 0-8, g 9 .. 9 + QT - 1
    const long long base = (long long)b * ny * nx;
    const long long n = base + (long long)y * nx + x;
    const C rho_ref = C(k.rho_ref);
    const C qdt = C(k.qdt);

    // temperature first: the Boussinesq force depends on it
    C e[QT], th = C(0);
    if (k.thermal) {
#pragma unroll
        for (int i = 0; i < QT; ++i) e[i] = C(A[bidx(npl, 9 + i, n)]);
        th = chan_th<QT, C>(e, qdt);
    }
    C ftx, fty;
    chan_force(k, th, ftx, fty);

    C d[9], drho, rho, ux, uy;
    chan_flow_macros<C, S>(A, npl, n, rho_ref, ftx, fty, d, drho, rho, ux, uy);
    C ds[9], es[QT];
    chan_collide<C, QT>(k, d, drho, rho, ux, uy, ftx, fty, e, th, qdt, ds, es);

    // ---- outlet wall velocity: 1.5 u(x_b) - 0.5 u(x_b - 1) at time t
    C uwx = C(0), uwy = C(0);
    const bool outlet = k.bcx == 1 && x == nx - 1;
    if (k.flow && outlet) {
        C d2[9], dr2, r2, ux2, uy2, fx2 = ftx, fy2 = fty;
        if (k.buoy) {  // the force of that node, as it computes it itself
            C e2[QT];
#pragma unroll
            for (int i = 0; i < QT; ++i) e2[i] = C(A[bidx(npl, 9 + i, n - 1)]);
            chan_force(k, chan_th<QT, C>(e2, qdt), fx2, fy2);
        }
        chan_flow_macros<C, S>(A, npl, n - 1, rho_ref, fx2, fy2, d2, dr2, r2, ux2, uy2);
        uwx = C(1.5) * ux - C(0.5) * ux2;
        uwy = C(1.5) * uy - C(0.5) * uy2;
    }

    // ---- streaming with boundary substitution (a frozen flow keeps its
    //      populations).  A population leaving through the symmetry plane
    //      re-enters as its mirror image at x + c_x (Eq. simetria); where that
    //      lies outside in x the x rule applies.
    if (!k.flow) {
#pragma unroll
        for (int i = 0; i < 9; ++i) B[bidx(npl, i, n)] = S(d[i]);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int tx = x + EX[i], ty = y + EY[i], j = i;
            const bool sym = k.bcy == 2 && ty >= ny;
            if (sym) {
                ty = ny - 1;
                j = MIRY[i];
            }
            const bool outy = k.bcy && !sym && (ty < 0 || ty >= ny);
            const bool outx = k.bcx && (tx < 0 || tx >= nx);
            if (!outy && !outx) {
                tx = wrap(tx, nx);
                ty = wrap(ty, ny);
                B[bidx(npl, j, base + (long long)ty * nx + tx)] = S(ds[i]);
            } else {
                C v;
                if (outy || k.bcx == 2)
                    v = ds[i];  // halfway bounce-back, Eq. BB_vel with u_w = 0
                else if (tx < 0)
                    v = chan_inlet_f<C>(i, ds[i], rho_ref, C(uin[y]));
                else
                    v = chan_outlet_f<C>(i, ds[i], rho_ref, uwx, uwy);
                B[bidx(npl, OPP[i], n)] = S(v);
            }
        }
    }
    if (k.thermal) {
        // Thermal outlet, first-order extrapolation g_j(x_b) = g_j(x_b - 1) at
        // t + dt: each value stored into column nx - 2 for a population with
        // c_x < 0 is stored into the outlet column as well, unless a wall rule
        // owns that outlet slot (its source lies beyond a wall in y).
        auto put = [&](int j, int tx, int ty, C v) {
            B[bidx(npl, 9 + j, base + (long long)ty * nx + tx)] = S(v);
            if (k.bcx == 1 && tx == nx - 2 && tex<QT>(j) < 0) {
                const int sy = ty - tey<QT>(j);
                const bool wall_owned = k.bcy && (sy < 0 || (k.bcy == 1 && sy >= ny));
                if (!wall_owned) B[bidx(npl, 9 + j, base + (long long)ty * nx + nx - 1)] = S(v);
            }
        };
#pragma unroll
        for (int i = 0; i < QT; ++i) {
            int tx = x + tex<QT>(i), ty = y + tey<QT>(i), j = i;
            const bool sym = k.bcy == 2 && ty >= ny;
            if (sym) {
                ty = ny - 1;
                j = tmir<QT>(i);
            }
            const bool outy = k.bcy && !sym && (ty < 0 || ty >= ny);
            const bool outx = k.bcx && (tx < 0 || tx >= nx);
            if (!outy && !outx) {
                put(j, wrap(tx, nx), wrap(ty, ny), es[i]);
            } else if (outy) {
                put(topp<QT>(i), x, y, chan_flux_g<QT, C>(i, es[i], C(qw[x]), C(mod)));
            } else if (k.bcx == 2) {
                // fixed-temperature side wall (App. D)
                put(topp<QT>(i), x, y, chan_antibb_g<QT, C>(i, es[i], C(k.Tw[tx < 0 ? 0 : 1])));
            } else if (tx < 0) {
                // anti-bounce-back Dirichlet inlet, T_w where the link crosses
                // the inlet (between rows y and y + c_y)
                const int y2 = y + tey<QT>(i);
                const C tw = (y2 >= 0 && y2 < ny) ? C(0.5) * (C(tin[y]) + C(tin[y2])) : C(tin[y]);
                put(topp<QT>(i), x, y, chan_antibb_g<QT, C>(i, es[i], tw));
            }
            // populations leaving through the outlet: the outlet slots are filled
            // by the extrapolation stores of put()
        }
    }
}

// ---------------------------------------------------------------------------
// Two channel steps per launch (temporal blocking) for flow with temperature
// (QT: the D2Q5 or D2Q9 thermal set; Boussinesq force optional), x periodic,
// inlet/outlet or fixed-temperature end walls and y periodic, walls, or a wall
// below and the symmetry plane above.  A workgroup of 256 lanes takes one x-tile of one
// row segment [a, e) of one replica: lane l holds column c = 252 t - 2 + l
// (modulo nx for periodic x; with x ends, lanes whose column lies outside
// [0, nx) read a clamped column and their results are never used).  At row v
// it collides step n at row v and step n + 1 at row v - 1:
//   - step n hands its x-moving post-collision values (and u, for the
//     outlet's wall velocity) to the neighbour lanes through LDS and
//     accumulates them into the step-(n + 1) state of rows v - 1, v and
//     v + 1, which stays in registers; row v - 1 is complete once row v has
//     collided;
//   - step n + 1 at row v - 1 pushes straight to memory with the streaming
//     and boundary rules of k_chan_step; its u reaches the next lane through
//     LDS for the outlet (a second barrier, inlet/outlet channels only).
// Step n is exact on every lane, the step-(n + 1) state on lanes 1..254 and
// the step-(n + 1) outlet velocity on lanes 2..254: lanes 2..253 store, so
// neighbouring tiles store disjoint columns.  Step n runs on rows a - 1 .. e
// (those that exist), step n + 1 on the segment's own rows, and every slot
// of the new state is written by its source node only.  Per node the
// arithmetic is that of k_chan_step (chan_th, chan_collide and the boundary
// values), so two steps here equal two single steps bit for bit.  mod0 and
// mod1 are the wall-flux modulations at t and t + dt.
// ALIGNED: nx a multiple of 64 and a row's node blocks under 2 GiB, so every
// row starts on a node block and an access is the row's block base (uniform)
// plus a 32-bit lane offset.  ENDS: the code for the cavity's end walls and
// the symmetry plane is compiled in (kept out of the other configurations:
// with it the 16384 x 2048 channel step took 0.462 ms instead of 0.419).
// ---------------------------------------------------------------------------
constexpr int kCtLanes = 256;
constexpr int kCtHalo = 2;                      // overlap columns per side
constexpr int kCtOut = kCtLanes - 2 * kCtHalo;  // stored columns per tile
// values per node (f 0-8, g from 9) and LDS exchange rows of step n (6 flow
// x movers, the thermal x movers 1 and 3, u, then the thermal diagonals 5-8)
constexpr int ct_nv(int qt) { return 9 + qt; }
constexpr int ct_x(int qt) { return qt == 9 ? 14 : 10; }

template <typename S, bool ALIGNED, bool ENDS, int QT>
__global__ __launch_bounds__(kCtLanes) void k_chan_tb2(ChanK k, const S* __restrict__ A,
                                                      S* __restrict__ B, const S* __restrict__ qw,
                                                      const S* __restrict__ uin,
                                                      const S* __restrict__ tin, S mod0, S mod1,
                                                      int seg) {
    using C = S;
    constexpr int NV = ct_nv(QT), G = 9, NX = ct_x(QT);
    const int nx = k.nx, ny = k.ny;
    const int nseg = (ny + seg - 1) / seg;
    const int ntx = (nx + kCtOut - 1) / kCtOut;
    int w;
    if (!xcd_tile(ntx * nseg * k.batch, w)) return;  // whole workgroup, before any barrier
    const int tx = w % ntx;  // x fastest
    w /= ntx;
    const int b = w / nseg;
    const int a = (w - b * nseg) * seg;
    const int e = min(a + seg, ny);
    const bool walls = k.bcy != 0;  // y ends: a wall at y-, a wall or the symmetry plane at y+
    const bool symy = ENDS && k.bcy == 2;  // the symmetry plane of Eq. simetria at y+
    const bool xends = k.bcx != 0;  // x not periodic: the channel has a left and a right end
    const bool io = ENDS ? k.bcx == 1 : xends;  // velocity inlet (left), pressure outlet (right)
    const bool xw = ENDS && k.bcx == 2;  // fixed-temperature no-slip walls at both ends
    const int s1 = walls ? max(a - 1, 0) : a - 1;   // first row of step n
    const int e1 = walls ? min(e + 1, ny) : e + 1;  // end of the step-n rows
    const long long base = (long long)b * ny * nx;
    const unsigned lx = threadIdx.x;
    const int col = tx * kCtOut - kCtHalo + int(lx);
    const unsigned x = unsigned(xends ? min(max(col, 0), nx - 1) : ((col % nx) + nx) % nx);
    const bool own = int(lx) >= kCtHalo && int(lx) < kCtLanes - kCtHalo && col < nx;
    const bool x_lo = xends && col == 0, x_hi = xends && col == nx - 1;  // the end columns
    const bool at_in = io && x_lo, at_out = io && x_hi;
    const unsigned xm = x == 0 ? nx - 1 : x - 1;
    const unsigned xp = x == unsigned(nx - 1) ? 0u : x + 1;
    const unsigned lxm = lx == 0 ? 0u : lx - 1;
    const unsigned lxp = lx == kCtLanes - 1 ? lx : lx + 1;
    const C rho_ref = C(k.rho_ref), qdt = C(k.qdt);
    const C q = C(qw[x]);
    const C tw_lo = C(k.Tw[0]), tw_hi = C(k.Tw[1]);

    __shared__ C xch[2][NX][kCtLanes];  // step n: x movers and u, rows v mod 2
    __shared__ C un1[2][2][kCtLanes];     // step n + 1: u, rows v mod 2

    // memory row of virtual row v: step-n rows of a periodic segment lie in
    // [-1, ny], so one correction wraps them
    auto rowof = [&](int v) { return v < 0 ? v + ny : (v >= ny ? v - ny : v); };
    // value i of the node in column slot c (0: x, 1: x - 1, 2: x + 1) of row v
    const unsigned xcol[3] = {x, xm, xp};
    unsigned boff[3];  // ALIGNED: byte offset of value 0 of those columns within a row
#pragma unroll
    for (int c = 0; c < 3; ++c)
        boff[c] = unsigned(((xcol[c] >> 6) * NV * kBlk + (xcol[c] & (kBlk - 1))) * sizeof(S));
    auto at = [&](auto* P, int v, int c, int i) {
        const long long ro = base + (long long)rowof(v) * nx;
        if constexpr (ALIGNED) {
            using B8 = std::conditional_t<std::is_const_v<std::remove_pointer_t<decltype(P)>>,
                                          const char, char>;
            auto* row = (B8*)P + (ro >> 6) * (long long)(NV * kBlk * sizeof(S));
            return (decltype(P))(row + boff[c]) + i * kBlk;
        } else {
            return P + bidx(NV, i, ro + xcol[c]);
        }
    };
    auto load_row = [&](int v, C (&s)[NV]) {
#pragma unroll
        for (int i = 0; i < NV; ++i) s[i] = C(*at(A, v, 0, i));
    };
    // macros and both collisions of one node, as in k_chan_step
    auto collide = [&](const C (&s)[NV], C& ux, C& uy, C (&ds)[9], C (&es)[QT]) {
        C d[9], g[QT], drho, rho, ftx, fty;
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = s[i];
#pragma unroll
        for (int i = 0; i < QT; ++i) g[i] = s[G + i];
        const C th = chan_th<QT, C>(g, qdt);
        chan_force(k, th, ftx, fty);
        chan_flow_macros_v<C>(d, rho_ref, ftx, fty, drho, rho, ux, uy);
        chan_collide<C, QT>(k, d, drho, rho, ux, uy, ftx, fty, g, th, qdt, ds, es);
    };

    // Register slots: slot (u - s1) mod 3 holds the accumulated step-(n + 1)
    // state of row u (rows v - 1 .. v + 1 are live).  The row loop is
    // unrolled three times, so every slot index is a compile-time constant.
    // The stored state of row v is read at the start of its own row step:
    // reading it a row ahead (in registers) took 6 % longer.
    C Ld[NV], Ac[3][NV];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < NV; ++i) Ac[j][i] = C(0);

    auto row_step = [&](int v, auto Jc) {
        constexpr int J = decltype(Jc)::value;
        constexpr int s0 = J, sn = (J + 1) % 3, sm1 = (J + 2) % 3;  // rows v, v + 1, v - 1
        const bool do_n = v < e1;
        // unconditional (the last row step re-reads an existing row)
        load_row(do_n ? v : e1 - 1, Ld);
        C(&xb)[NX][kCtLanes] = xch[v & 1];
        // ---- step n at row v
        C ds[9], es[QT], ux = C(0), uy = C(0);
        if (do_n) {
            collide(Ld, ux, uy, ds, es);
            xb[0][lx] = ds[1];
            xb[1][lx] = ds[3];
            xb[2][lx] = ds[5];
            xb[3][lx] = ds[6];
            xb[4][lx] = ds[7];
            xb[5][lx] = ds[8];
            xb[6][lx] = es[1];
            xb[7][lx] = es[3];
            if constexpr (QT == 9) {
                xb[10][lx] = es[5];
                xb[11][lx] = es[6];
                xb[12][lx] = es[7];
                xb[13][lx] = es[8];
            }
            xb[8][lx] = ux;
            xb[9][lx] = uy;
        }
        __syncthreads();  // the other buffer's reads ended a row ago
        if (do_n) {
            // pushes of row v: rest and x movers to row v, +y movers to row
            // v + 1, -y movers to row v - 1 (x movers from the lanes x -+ 1)
            C(&A0)[NV] = Ac[s0];
            C(&Ap)[NV] = Ac[sn];
            C(&A1)[NV] = Ac[sm1];
            const bool top = k.bcy == 1 && v == ny - 1, bottom = walls && v == 0;
            const bool stop = symy && v == ny - 1;  // top row under the symmetry plane
            C uwx = C(0), uwy = C(0), u_in = C(0), t_in = C(0);
            if (io) {
                const int y = rowof(v);
                u_in = C(uin[y]);
                t_in = C(0.5) * (C(tin[y]) + C(tin[y]));  // the inlet link stays in row y
                uwx = C(1.5) * ux - C(0.5) * xb[8][lxm];
                uwy = C(1.5) * uy - C(0.5) * xb[9][lxm];
            }
            // an end wall (xw) bounces back like the y walls (u_w = 0)
            A0[0] = ds[0];
            A0[1] = x_lo ? (io ? chan_inlet_f<C>(3, ds[3], rho_ref, u_in) : ds[3]) : xb[0][lxm];
            A0[3] = x_hi ? (io ? chan_outlet_f<C>(1, ds[1], rho_ref, uwx, uwy) : ds[1])
                         : xb[1][lxp];
            // the -y slots take the top wall's values; below the top row the
            // next row's pushes overwrite them (not the inlet's and outlet's
            // own values)
            A0[4] = ds[2];
            A0[7] = at_out && !top ? chan_outlet_f<C>(5, ds[5], rho_ref, uwx, uwy) : ds[5];
            A0[8] = at_in && !top ? chan_inlet_f<C>(6, ds[6], rho_ref, u_in) : ds[6];
            // under the symmetry plane the +y movers come back mirrored at
            // x + c_x (Eq. simetria), from the neighbour lanes
            A0[7] = stop && !x_hi ? xb[3][lxp] : A0[7];
            A0[8] = stop && !x_lo ? xb[2][lxm] : A0[8];
            // the +y slots hold the row below's pushes, except at the bottom
            // wall and where the source lies beyond an x end
            A0[2] = bottom ? ds[4] : A0[2];
            A0[5] = bottom ? ds[7]
                           : (x_lo ? (io ? chan_inlet_f<C>(7, ds[7], rho_ref, u_in) : ds[7])
                                   : A0[5]);
            A0[6] = bottom ? ds[8]
                           : (x_hi ? (io ? chan_outlet_f<C>(8, ds[8], rho_ref, uwx, uwy) : ds[8])
                                   : A0[6]);
            Ap[2] = ds[2];
            Ap[5] = xb[2][lxm];
            Ap[6] = xb[3][lxp];
            A1[4] = ds[4];
            A1[7] = x_hi ? A1[7] : xb[4][lxp];
            A1[8] = x_lo ? A1[8] : xb[5][lxm];
            // temperature: Dirichlet inlet or end walls (anti-bounce-back),
            // outlet extrapolation (the value its left neighbour receives:
            // the outlet node's own), flux walls
            if constexpr (QT == 5) {
                A0[G + 0] = es[0];
                A0[G + 1] = x_lo ? chan_antibb_g<QT, C>(3, es[3], io ? t_in : tw_lo) : xb[6][lxm];
                A0[G + 3] = x_hi ? (io ? es[3] : chan_antibb_g<QT, C>(1, es[1], tw_hi)) : xb[7][lxp];
                A0[G + 4] = stop ? es[2] : chan_flux_g<QT, C>(2, es[2], q, mod0);
                A0[G + 2] = bottom ? chan_flux_g<QT, C>(4, es[4], q, mod0) : A0[G + 2];
                Ap[G + 2] = es[2];
                A1[G + 4] = es[4];
            } else {
                // D2Q9 thermal set: the diagonals follow the flow's pattern.
                // Inlet temperature where a link crosses the inlet: the mean
                // of its two rows (the row's own value if the other is beyond
                // the channel).
                C tw6 = C(0), tw7 = C(0);
                if (io) {
                    const int y = rowof(v);
                    tw6 = y + 1 < ny ? C(0.5) * (C(tin[y]) + C(tin[y + 1])) : C(tin[y]);
                    tw7 = y - 1 >= 0 ? C(0.5) * (C(tin[y]) + C(tin[y - 1])) : C(tin[y]);
                }
                const C l8 = chan_antibb_g<QT, C>(6, es[6], io ? tw6 : tw_lo);
                const C l5 = chan_antibb_g<QT, C>(7, es[7], io ? tw7 : tw_lo);
                A0[G + 0] = es[0];
                A0[G + 1] = x_lo ? chan_antibb_g<QT, C>(3, es[3], io ? t_in : tw_lo) : xb[6][lxm];
                A0[G + 3] = x_hi ? (io ? es[3] : chan_antibb_g<QT, C>(1, es[1], tw_hi)) : xb[7][lxp];
                // -y slots: top wall flux, mirrored movers under the symmetry
                // plane, else provisional (the row above overwrites them, but
                // not the end columns' own values)
                A0[G + 4] = stop ? es[2] : chan_flux_g<QT, C>(2, es[2], q, mod0);
                A0[G + 7] = top ? chan_flux_g<QT, C>(5, es[5], q, mod0)
                          : x_hi ? (io ? es[6] : chan_antibb_g<QT, C>(5, es[5], tw_hi))
                                 : xb[11][lxp];
                A0[G + 8] = top ? chan_flux_g<QT, C>(6, es[6], q, mod0) : x_lo ? l8 : xb[10][lxm];
                // +y slots: bottom wall flux, the end columns' own values
                A0[G + 2] = bottom ? chan_flux_g<QT, C>(4, es[4], q, mod0) : A0[G + 2];
                A0[G + 5] = bottom ? chan_flux_g<QT, C>(7, es[7], q, mod0) : x_lo ? l5 : A0[G + 5];
                A0[G + 6] = bottom ? chan_flux_g<QT, C>(8, es[8], q, mod0)
                          : (x_hi && xw) ? chan_antibb_g<QT, C>(8, es[8], tw_hi) : A0[G + 6];
                Ap[G + 2] = es[2];
                Ap[G + 5] = xb[10][lxm];
                Ap[G + 6] = at_out ? es[6] : xb[11][lxp];
                A1[G + 4] = es[4];
                A1[G + 7] = (x_hi && xw) ? A1[G + 7] : at_out ? es[7] : xb[12][lxp];
                A1[G + 8] = x_lo ? A1[G + 8] : xb[13][lxm];
            }
        }
        // ---- step n + 1 at row r = v - 1, complete now, straight to memory
        const int r = v - 1;
        const bool do_n1 = r >= a && r < e;
        C ds1[9], es1[QT], ux1 = C(0), uy1 = C(0);
        if (do_n1) {
            collide(Ac[sm1], ux1, uy1, ds1, es1);
            if (io) {
                un1[v & 1][0][lx] = ux1;
                un1[v & 1][1][lx] = uy1;
            }
        }
        if (io) __syncthreads();
        if (do_n1 && own) {
            C uwx = C(0), uwy = C(0), u_in = C(0), t_in = C(0);
            if (io) {
                u_in = C(uin[r]);
                t_in = C(0.5) * (C(tin[r]) + C(tin[r]));
                uwx = C(1.5) * ux1 - C(0.5) * un1[v & 1][0][lxm];
                uwy = C(1.5) * uy1 - C(0.5) * un1[v & 1][1][lxm];
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int ty = r + EY[i];
                // under the symmetry plane a +y mover comes back mirrored into the
                // top row (a separate branch keeps every value index a constant)
                const bool sym = symy && ty >= ny;
                const bool outy = walls && !sym && (ty < 0 || ty >= ny);
                const bool outx = (EX[i] < 0 && x_lo) || (EX[i] > 0 && x_hi);
                if (sym && !outx) {
                    st(at(B, r, EX[i] == 0 ? 0 : (EX[i] > 0 ? 2 : 1), MIRY[i]), S(ds1[i]));
                } else if (!outy && !outx) {
                    st(at(B, ty, EX[i] == 0 ? 0 : (EX[i] > 0 ? 2 : 1), i), S(ds1[i]));
                } else {
                    C val;
                    if (outy || xw)
                        val = ds1[i];
                    else if (EX[i] < 0)
                        val = chan_inlet_f<C>(i, ds1[i], rho_ref, u_in);
                    else
                        val = chan_outlet_f<C>(i, ds1[i], rho_ref, uwx, uwy);
                    st(at(B, r, 0, OPP[i]), S(val));
                }
            }
#pragma unroll
            for (int i = 0; i < QT; ++i) {
                const int cx = tex<QT>(i), cy = tey<QT>(i);
                const int ty = r + cy;
                const bool sym = symy && ty >= ny;
                const bool outy = walls && !sym && (ty < 0 || ty >= ny);
                const bool outx = (cx < 0 && x_lo) || (cx > 0 && x_hi);
                const int col = cx == 0 ? 0 : (cx > 0 ? 2 : 1);
                // outlet extrapolation: what column nx - 2 receives in a slot
                // with c_x < 0 (never a slot a wall rule owns here: its
                // source is this row or, mirrored, the row itself)
                if (sym && !outx) {
                    st(at(B, r, col, G + tmir<QT>(i)), S(es1[i]));
                    if (tex<QT>(tmir<QT>(i)) < 0 && at_out) st(at(B, r, 0, G + tmir<QT>(i)), S(es1[i]));
                } else if (!outy && !outx) {
                    st(at(B, ty, col, G + i), S(es1[i]));
                    if (cx < 0 && at_out) st(at(B, ty, 0, G + i), S(es1[i]));
                } else if (outy) {
                    st(at(B, r, 0, G + topp<QT>(i)), S(chan_flux_g<QT, C>(i, es1[i], q, mod1)));
                } else if (xw) {
                    st(at(B, r, 0, G + topp<QT>(i)),
                       S(chan_antibb_g<QT, C>(i, es1[i], cx < 0 ? tw_lo : tw_hi)));
                } else if (cx < 0) {
                    // the inlet temperature where the link crosses the inlet
                    const int y2 = r + cy;
                    const C tw = cy == 0 ? t_in
                               : (y2 >= 0 && y2 < ny) ? C(0.5) * (C(tin[r]) + C(tin[y2]))
                                                      : C(tin[r]);
                    st(at(B, r, 0, G + topp<QT>(i)), S(chan_antibb_g<QT, C>(i, es1[i], tw)));
                }
                // the outlet's own +x movers leave; their slots are extrapolated
            }
        }
    };
    const int vend = e + 1;
    for (int v = s1; v < vend; v += 3) {
        row_step(v, std::integral_constant<int, 0>{});
        if (v + 1 >= vend) break;
        row_step(v + 1, std::integral_constant<int, 1>{});
        if (v + 2 >= vend) break;
        row_step(v + 2, std::integral_constant<int, 2>{});
    }
}

// ---------------------------------------------------------------------------
// Two-phase model: conservative Allen-Cahn h_i (BGK) + pressure z_i (MRT/BGK)
// State planes (node-block layout, PhasePlanes): 0-8 h_i, 9-17 z_i, then
// (FP32 storage only) the low part of h_0, then (phi u) of the previous step
// (2 planes): npop = 19 (FP32) or 18 (FP64) population planes plus 2.
// ---------------------------------------------------------------------------

#ifndef LBM_PHASE_TY
#define LBM_PHASE_TY 8
#endif
constexpr int TX = 64, TY = LBM_PHASE_TY;
// LDS reserved by each FP32 single-step workgroup beyond its own ~1.5 KB: it
// holds residency at four 256-thread workgroups per CU (4 waves per SIMD).
// With more waves resident, more of the 42 population streams per wave are
// open in DRAM at once and the step runs slower (67M-node bubble batch:
// 2.82 ms at 8 waves per SIMD, 2.56 ms at 4).  The FP64 kernel's register
// use already gives 4 waves per SIMD.
constexpr unsigned kPhaseLdsReserve = 36864;
// Planes of the two-phase D2Q9 state in the node-block layout (bidx): h_0..h_8,
// z_0..z_8, in FP32 the low part of h_0, then (phi u)_x and (phi u)_y.
template <typename S>
struct PhasePlanes {
    static constexpr bool RMASS = std::is_same<S, float>::value;
    static constexpr int NPL = RMASS ? 21 : 20;
    static constexpr int H = 0, Z = 9, LO = 18, PU = RMASS ? 19 : 18;
};
template <typename S>
__device__ __forceinline__ long long pidx(int i, long long n) {
    return bidx(PhasePlanes<S>::NPL, i, n);
}

// phi of a node from its stored h_i, Eq. zero_moment_h (rest population with
// its low part).  One summation order everywhere, so that every kernel sees
// the same phi for the same populations.
template <typename C>
__device__ __forceinline__ C phi_sum(const C (&h)[9], C hlo) {
    return (h[0] + hlo) + (((h[1] + h[3]) + (h[2] + h[4])) + ((h[5] + h[7]) + (h[6] + h[8])));
}

// Reciprocals of the two-phase collision: the hardware's 1-ulp reciprocal and
// reciprocal square root in FP32 (FP32 storage carries ~1e-7 relative
// rounding anyway), exact division in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// Everything a node derives from its phi neighbourhood and its z_i before
// the collision.  pn[i] = phi at x + e_i (pn[0] = phi at the node).
template <typename C>
struct PhaseLocal {
    C phi, Gx, Gy, rho, drl, wn, mu, fsx, fsy, nxv, nyv, ux, uy, uu, ug, ph;
};

template <typename C>
__device__ __forceinline__ PhaseLocal<C> phase_local(const PhaseK& k, const C (&pn)[9],
                                                     const C (&z)[9]) {
    PhaseLocal<C> L;
    // ---- stencils, Eq. gradient and Eq. laplacian in lattice form:
    //      grad phi = 3 G / dx, lap phi = 6 L / dx^2 with G = sum w_i e_i phi_i and
    //      L = sum w_i (phi_i - phi), summed by weight class (1/9 on the axes,
    //      1/36 on the diagonals).  Both are built from differences of
    //      neighbouring values, which are exact in floating point; a sum of the
    //      neighbours minus (5/9) phi would cancel terms of size phi down to the
    //      Laplacian and lose most of its digits in FP32.
    const C phi = pn[0];
    const C dpp = pn[5] - pn[7];  // (+1,+1) - (-1,-1)
    const C dpm = pn[8] - pn[6];  // (+1,-1) - (-1,+1)
    const C Gx = C(1.0 / 9.0) * (pn[1] - pn[3]) + C(1.0 / 36.0) * (dpp + dpm);
    const C Gy = C(1.0 / 9.0) * (pn[2] - pn[4]) + C(1.0 / 36.0) * (dpp - dpm);
    const C sax = ((pn[1] - phi) + (pn[3] - phi)) + ((pn[2] - phi) + (pn[4] - phi));
    const C sdg = ((pn[5] - phi) + (pn[7] - phi)) + ((pn[6] - phi) + (pn[8] - phi));
    const C Lp = C(1.0 / 9.0) * sax + C(1.0 / 36.0) * sdg;
    const C drl = C(k.rho_l - k.rho_g);
    const C rho = C(k.rho_g) + phi * drl;  // linear in phi (Sec. 2.3)
    const C ir = rcp(rho);
    // dt / tau = 1 / (3 nu dt / dx^2 + 1/2), with nu linear in phi or, in the
    // zeta form of Sec. 4.4, nu = zeta / rho
    if (k.visc_mode == 0) {
        L.wn = rcp(C(3) * (C(k.nuh_g) + phi * C(k.nuh_l - k.nuh_g)) + C(0.5));
    } else {
        const C zh = C(k.zh_g) + phi * C(k.zh_l - k.zh_g);
        L.wn = rho * rcp(C(3) * zh + C(0.5) * rho);
    }
    // chemical potential, Eq. chemical_potential; surface force F_s = mu grad phi
    const C mu = C(4) * C(k.beta) * phi * (phi - C(1)) * (phi - C(0.5)) - C(k.kap6) * Lp;
    L.fsx = mu * Gx * C(k.fs_scale) + C(k.Fbt[0]);
    L.fsy = mu * Gy * C(k.fs_scale) + C(k.Fbt[1]);
    // guarded interface normal (text after Eq. laplacian)
    const C gn2 = Gx * Gx + Gy * Gy;
    L.nxv = C(0);
    L.nyv = C(0);
    if (gn2 > C(k.Geps) * C(k.Geps)) {
        const C ig = rsq(gn2);
        L.nxv = Gx * ig;
        L.nyv = Gy * ig;
    }
    // ---- pressure populations: velocity first (Eq. u_Liang), then pressure
    const C jx = (z[1] - z[3]) + ((z[5] - z[7]) + (z[8] - z[6]));
    const C jy = (z[2] - z[4]) + ((z[5] - z[7]) + (z[6] - z[8]));
    L.ux = (jx + C(0.5) * L.fsx) * ir;
    L.uy = (jy + C(0.5) * L.fsy) * ir;
    L.uu = L.ux * L.ux + L.uy * L.uy;
    L.ug = L.ux * Gx + L.uy * Gy;
    const C zs = ((z[1] + z[3]) + (z[2] + z[4])) + ((z[5] + z[7]) + (z[6] + z[8]));
    // p / c_s^2, Eq. p_Liang: c_s^2/(1 - w_0) [sum_{i>0} z_i + dt/2 u.grad rho + rho s_0(u)]
    L.ph = C(1.8) * (zs + C(1.5) * drl * L.ug - C(1.5) * wgt<C>(0) * rho * L.uu);
    L.phi = phi;
    L.Gx = Gx;
    L.Gy = Gy;
    L.rho = rho;
    L.drl = drl;
    L.mu = mu;
    return L;
}

// The collision of one node.  In: its stored h_i (with the low part of h_0
// for FP32 storage), z_i, (phi u) of the previous step and its PhaseLocal.
// Out: post-collision h_i* (i > 0, in hs), h_0* as a hi/lo pair, z_i*, and
// the node's (phi u).
template <typename S, typename C>
__device__ __forceinline__ void phase_collide(const PhaseK& k, const PhaseLocal<C>& L,
                                              const C (&h)[9], C hlo, const C (&z)[9], C pu0,
                                              C pu1, C (&hs)[9], S& h0hi, S& h0lo, C (&zst)[9],
                                              C& pux, C& puy) {
    constexpr bool RMASS = std::is_same<S, float>::value;
    const C phi = L.phi, ux = L.ux, uy = L.uy;
    // ---- interface populations (Eq. eq_lattice_boltzmann_interface,
    //      source_term_interface, heq_liang); d(phi u)/dt by explicit Euler
    pux = phi * ux;
    puy = phi * uy;
    const C dpx = pux - pu0, dpy = puy - pu1;
    const C wphi = C(k.w_phi);
    const C sfac = C(1) - C(0.5) * wphi;
    const C sharp = C(4) * phi * (C(1) - phi) * C(k.dxW);
    // h_i* = h_i - w (h_i - h_i^eq) + S_i with h_i^eq = phi w_i (1 + 3 e_i.u) and
    // S_i = (1 - w/2) w_i e_i.(3 d(phi u) + sharp n) collects into
    //   h_i* = h_i + (t_i - w h_i),  t_i = w_i (a + e_i.B),
    //   a = w phi,  B = 3 w phi u + (1 - w/2)(3 d(phi u) + sharp n);
    // t_i - w h_i is the step's small change, taken in one fused multiply-add
    // (one rounding of the change, as the non-equilibrium form has).
    const C a = wphi * phi;
    const C a3 = C(3) * a;
    const C Bx = a3 * ux + sfac * (C(3) * dpx + sharp * L.nxv);
    const C By = a3 * uy + sfac * (C(3) * dpy + sharp * L.nyv);
    const C qa = C(1.0 / 9.0) * a, qx = C(1.0 / 9.0) * Bx, qy = C(1.0 / 9.0) * By;
    const C da = C(1.0 / 36.0) * a, ds = C(1.0 / 36.0) * (Bx + By), dd = C(1.0 / 36.0) * (Bx - By);
    const C t[9] = {C(4.0 / 9.0) * a, qa + qx, qa + qy, qa - qx, qa - qy,  // 0, (+1,0) (0,+1) (-1,0) (0,-1)
                    da + ds, da - dd, da - ds, da + dd};                   // (+1,+1) (-1,+1) (-1,-1) (+1,-1)
    hs[0] = C(0);
#pragma unroll
    for (int i = 1; i < 9; ++i) hs[i] = h[i] + (t[i] - wphi * h[i]);
    h0lo = S(0);
    if constexpr (RMASS) {
        // rest population takes the node's exact balance: h0* = phi - sum_{i>0} h_i*
        // with the stored (rounded) h_i*.  The FP32 terms are summed in FP64
        // (each exact there; 18 terms lose at most ~2^-49 of the largest) and
        // the sum is kept as an FP32 hi/lo pair.
        double acc = double(h[0]) + double(hlo);
#pragma unroll
        for (int i = 1; i < 9; ++i) acc += double(h[i]);
#pragma unroll
        for (int i = 1; i < 9; ++i) acc -= double(float(hs[i]));
        h0hi = float(acc);
        h0lo = float(acc - double(h0hi));
    } else {
        h0hi = S(h[0] + (t[0] - wphi * h[0]));  // h_0^eq = (4/9) phi, no source
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
    const C rho = L.rho, drl = L.drl, wn = L.wn, Gx = L.Gx, Gy = L.Gy;
    const C ruu = rho * L.uu, D = drl * L.ug;
    const C meq[9] = {C(0), C(2) * L.ph + C(3) * ruu, C(-3) * (L.ph + ruu), rho * ux, -rho * ux,
                      rho * uy, -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy};
    const C mf[9] = {C(3) * D, C(0), C(-3) * D, L.fsx, -L.fsx, L.fsy, -L.fsy,
                     C(2) * drl * (Gx * ux - Gy * uy), drl * (Gx * uy + Gy * ux)};
    C m[9];
    if (k.z_mrt) {
        // Sec. 3 rates: rho, e, eps, j_x, j_y relax at 1/dt, which leaves
        // m* = m^eq + m^F / 2 whatever the incoming moment; q_x and q_y relax at
        // w_q (q_y at 1/dt in the printed variant), the stresses at w_nu.  Only
        // the moments of those four rows are taken from z.
        const C x13 = z[1] - z[3], y24 = z[2] - z[4];
        const C x58 = (z[5] - z[7]) + (z[8] - z[6]);
        const C y58 = (z[5] - z[7]) + (z[6] - z[8]);
        const C wq = C(3) * (C(2) - wn) * rcp(C(3) - wn);
        const C wqy = k.qy_printed ? C(1) : wq;
        const C mq[4] = {C(-2) * x13 + x58, C(-2) * y24 + y58, (z[1] + z[3]) - (z[2] + z[4]),
                         (z[5] + z[7]) - (z[6] + z[8])};
        const C Lq[4] = {wq, wqy, wn, wn};
        const int row[4] = {4, 6, 7, 8};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = row[j];
            m[q] = mq[j] - Lq[j] * (mq[j] - meq[q]) + (C(1) - C(0.5) * Lq[j]) * mf[q];
        }
        m[0] = meq[0] + C(0.5) * mf[0];
        m[1] = meq[1];  // m^F has no e component
        m[2] = meq[2] + C(0.5) * mf[2];
        m[3] = meq[3] + C(0.5) * mf[3];
        m[5] = meq[5] + C(0.5) * mf[5];
    } else {
        // BGK: every row at dt / tau
        moments9(z, m);
#pragma unroll
        for (int q = 0; q < 9; ++q) m[q] += -wn * (m[q] - meq[q]) + (C(1) - C(0.5) * wn) * mf[q];
    }
    inverse9(m, zst);
}

// ---------------------------------------------------------------------------
// Single step.  Tile of TX x TY nodes per block (64 x 8, or nx x 512/nx for
// replicas narrower than 64 nodes, so that no lane idles and a wave still
// covers 64 contiguous nodes); phi of the tile and a one-node ring in LDS.
// MACROS: evaluate the macroscopic fields of the stored state into mout
// instead of stepping.
// ---------------------------------------------------------------------------
// One tile of the single step (every thread of the block calls it; it has
// one barrier).  Returns early for threads without a node, after the barrier.
template <typename S, typename C, bool MACROS, int TX, int TY>
__device__ __forceinline__ void phase_tile(const PhaseK& k, int tile, const S* __restrict__ A,
                                           S* __restrict__ B, double* __restrict__ mout,
                                           C (&sphi)[TY + 2][TX + 2]) {
    constexpr bool RMASS = std::is_same<S, float>::value;
    using PL = PhasePlanes<S>;
    const int nx = k.nx, ny = k.ny;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int gx = (nx + TX - 1) / TX, gy = (ny + TY - 1) / TY;
    const int b = tile / (gx * gy), r = tile - b * gx * gy;
    const int x0 = (r % gx) * TX, y0 = (r / gx) * TY;
    const long long base = (long long)b * ny * nx;
    auto gxw = [&](int gx) { return ((gx % nx) + nx) % nx; };
    auto gyw = [&](int gy) {
        if (k.bcy) return gy < 0 ? 0 : (gy >= ny ? ny - 1 : gy);  // mirror ghost at walls
        return ((gy % ny) + ny) % ny;
    };
    // Every load of the tile is issued before the barrier: the node's own h, z
    // and (phi u) (kept in registers for the collision) and, for 148 threads,
    // the 10 values of one ring node; the barrier then waits for memory once.
    const int x = x0 + tx, y = y0 + ty;
    const bool valid = x < nx && y < ny;
    const long long n = base + (long long)gyw(y) * nx + gxw(x);  // == own node when valid
    C h[9], z[9], hlo = C(0), pu0 = C(0), pu1 = C(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = C(A[pidx<S>(PL::H + i, n)]);
    if (RMASS) hlo = C(A[pidx<S>(PL::LO, n)]);
    if (valid) {
#pragma unroll
        for (int i = 0; i < 9; ++i) z[i] = C(A[pidx<S>(PL::Z + i, n)]);
        if constexpr (!MACROS) {
            pu0 = C(A[pidx<S>(PL::PU, n)]);
            pu1 = C(A[pidx<S>(PL::PU + 1, n)]);
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
        C hr[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) hr[i] = C(A[pidx<S>(PL::H + i, nn)]);
        ring = phi_sum(hr, RMASS ? C(A[pidx<S>(PL::LO, nn)]) : C(0));
    }
    sphi[ty + 1][tx + 1] = phi_sum(h, hlo);
    if (hx > -2) sphi[hy + 1][hx + 1] = ring;
    __syncthreads();
    if (!valid) return;

    C pn[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) pn[i] = sphi[ty + 1 + EY[i]][tx + 1 + EX[i]];
    const PhaseLocal<C> L = phase_local(k, pn, z);

    if constexpr (MACROS) {
        const long long Q = k.P;
        mout[0 * Q + n] = double(L.rho);
        mout[1 * Q + n] = double(L.ph) * k.cs2;
        mout[2 * Q + n] = double(L.ux) * k.c;
        mout[3 * Q + n] = double(L.uy) * k.c;
        mout[4 * Q + n] = 0.0;
        mout[5 * Q + n] = double(L.phi);
        mout[6 * Q + n] = double(L.mu);
        return;
    } else {
        C hs[9], zst[9], pux, puy;
        S h0hi, h0lo;
        phase_collide<S, C>(k, L, h, hlo, z, pu0, pu1, hs, h0hi, h0lo, zst, pux, puy);
        st(B + pidx<S>(PL::PU, n), S(pux));
        st(B + pidx<S>(PL::PU + 1, n), S(puy));
        // ---- streaming of h and z: x periodic; y periodic or halfway
        //      bounce-back walls
        st(B + pidx<S>(PL::H, n), h0hi);
        if constexpr (RMASS) st(B + pidx<S>(PL::LO, n), h0lo);
        st(B + pidx<S>(PL::Z, n), S(zst[0]));
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int tyd = y + EY[i];
            if (k.bcy && (tyd < 0 || tyd >= ny)) {
                st(B + pidx<S>(PL::H + OPP[i], n), S(hs[i]));
                st(B + pidx<S>(PL::Z + OPP[i], n), S(zst[i]));
            } else {
                const long long d = base + (long long)wrap(tyd, ny) * nx + wrap(x + EX[i], nx);
                st(B + pidx<S>(PL::H + i, d), S(hs[i]));
                st(B + pidx<S>(PL::Z + i, d), S(zst[i]));
            }
        }
    }
}

template <typename S, typename C, bool MACROS, int TX = lbm::TX, int TY = lbm::TY>
__global__ __launch_bounds__(TX * TY) void k_phase(PhaseK k, const S* __restrict__ A,
                                               S* __restrict__ B, double* __restrict__ mout) {
    static_assert(2 * (TX + 2) + 2 * TY <= TX * TY, "the ring must fit in one pass of the block");
    __shared__ C sphi[TY + 2][TX + 2];
    const int gx = (k.nx + TX - 1) / TX, gy = (k.ny + TY - 1) / TY;
    int tile;
    if (!xcd_tile(gx * gy * k.batch, tile)) return;  // whole workgroup, before any barrier
    phase_tile<S, C, MACROS, TX, TY>(k, tile, A, B, mout, sphi);
}

// ---------------------------------------------------------------------------
// Many steps in one launch for grids of a few tiles (the paper's C4 channel is
// 4 x 512 nodes: sixteen 4 x 32 tiles).  One workgroup per tile, all resident
// at once (cooperative launch).  Between steps a tile waits only for the
// tiles that, in the previous step, pushed into the nodes it reads or read
// the nodes its next pushes overwrite (the tiles around it; every tile of
// its replica when a ragged tail is one node thick), through per-tile step
// counters with device-scope release / acquire; a grid-wide barrier costs
// several times more on this GPU.  Every wait is bounded: past the bound the workgroup
// flags an error and leaves, and so do its neighbours in turn, so the grid
// always drains.  The per-tile work is phase_tile, as in k_phase, so the
// states agree with single-step launches to the last bit.
// ---------------------------------------------------------------------------
constexpr unsigned kPersistSpin = 1u << 22;  // polls before a wait counts as failed

template <typename S, typename C, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void k_phase_persist(PhaseK k, S* __restrict__ A,
                                                           S* __restrict__ B, int nsteps,
                                                           unsigned epoch0,
                                                           unsigned* __restrict__ flags,
                                                           unsigned* __restrict__ err) {
    static_assert(2 * (TX + 2) + 2 * TY <= TX * TY, "the ring of a tile needs a thread per node");
    __shared__ C sphi[TY + 2][TX + 2];
    __shared__ int bad;
    const int gx = (k.nx + TX - 1) / TX, gy = (k.ny + TY - 1) / TY;
    const int tile = blockIdx.x;
    const int b = tile / (gx * gy), r = tile - b * gx * gy;
    const int bx = r % gx, by = r / gx;
    // Tiles whose step s - 1 must be complete before this tile's step s: those
    // that write the tile's nodes or its ring in step s - 1 (data it reads) and
    // those that read, in step s - 1, the nodes it writes in step s.  When
    // every tile spans at least two nodes in x and y these are the tiles of the
    // same replica within one node (x periodic, y periodic or closed by
    // walls); a one-node ragged tail reaches further, and then the tile waits
    // for every tile of its replica.
    const bool thin = (gx > 1 && k.nx - (gx - 1) * TX < 2) || (gy > 1 && k.ny - (gy - 1) * TY < 2);
    const int lin = threadIdx.y * TX + threadIdx.x;
    // Lanes of the first wave watch one tile each: lane j < 8 the j-th of
    // the eight surrounding tiles (x wraps; y wraps unless walls close it),
    // or, for a one-node tail, lane j tile j of the replica (at most 64).
    int wt = -1;
    if (thin) {
        if (lin < gx * gy && lin != r) wt = lin;
    } else if (lin < 8) {
        const int j = lin < 4 ? lin : lin + 1;  // skip the centre of the 3 x 3 block
        const int ox = j % 3 - 1, oy = j / 3 - 1;
        int ty_ = by + oy;
        const bool outside = ty_ < 0 || ty_ >= gy;
        ty_ = (ty_ + gy) % gy;
        const int t = ty_ * gx + (bx + ox + gx) % gx;
        if (!(outside && k.bcy) && t != r) wt = t;
    }
    const bool watch = wt >= 0;
    const unsigned* wflag = flags + b * gx * gy + (watch ? wt : 0);
    if (lin == 0) bad = 0;
    for (int s = 0; s < nsteps; ++s) {
        if (s > 0 && lin < 64) {
            const unsigned want = epoch0 + unsigned(s);
            unsigned spins = 0;
            bool fail = false;
            for (;;) {
                // modular comparison: the counter is behind want
                const bool behind =
                    watch && __hip_atomic_load(wflag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                                     want > 0x7fffffffu;
                if (!__any(behind)) break;
                if (++spins > kPersistSpin ||
                    __any(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                    fail = true;
                    break;
                }
            }
            if (fail && lin == 0) {
                bad = 1;
                __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            // one acquire for the workgroup: its waves share this CU's caches
            // and follow the first wave through the barrier below
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (bad) return;  // uniform: every thread read it after the barrier
        const S* a = (s & 1) ? B : A;
        S* o = (s & 1) ? A : B;
        phase_tile<S, C, false, TX, TY>(k, tile, a, o, (double*)nullptr, sphi);
        // Every wave waits until its stores have reached the L2 (vmcnt counts
        // stores on this GPU), the barrier orders them before the first
        // lane's device-scope release, whose L2 write-back then carries the
        // whole tile: one write-back per workgroup and step instead of one
        // per wave.
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (lin == 0)
            __hip_atomic_store(&flags[tile], epoch0 + unsigned(s + 1), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Two steps per launch (temporal blocking).  A workgroup of nx threads (one
// per column, nx a multiple of 64 up to 256) marches up the rows of one
// segment [a, e) of one replica (rows per segment: phase_tb2_seg).  At row
// v it collides step n at row v and
// step n + 1 at row v - 3:
//   - the post-collision values of step n are exchanged in x through LDS and
//     accumulated, per column, into the step-(n + 1) state of rows v - 1, v
//     and v + 1, which stays in registers (a row's state is complete once
//     the row above it has collided);
//   - step n + 1 at row r needs phi_{n+1} of rows r - 1 .. r + 1, i.e. the
//     step-n collisions of rows r - 2 .. r + 2, hence the lag;
//   - phi of both steps lives in LDS rings of four rows.
// Only the state at n and at n + 2 touches memory: half the traffic of two
// single steps.  Periodic y: step n also collides the two rows on each side
// of the segment (their outputs feed only this workgroup's registers), so
// every segment is independent.  Walls: rows outside [0, ny) do not exist
// and the bounce-back of the single step applies at both walls.  The
// arithmetic per node is phase_local + phase_collide, as in k_phase.
//
// TILED: the same march for rows of any width, in x-tiles of 256 lanes that
// overlap by 3 columns on each side (the segment overlap of y applied in
// x).  Lane l of tile t holds column x0 - 3 + l (mod nx), x0 = 250 t; x
// neighbours in LDS are lanes l -+ 1, so step n is exact on lanes 1..254
// (phi_n of both neighbours), the step-(n + 1) state on lanes 2..253 (pushes
// from both neighbours), and step n + 1 on lanes 3..252 (phi_{n+1} of both
// neighbours): those 250 columns are stored, the edge lanes' values are
// never used.  The stored columns of neighbouring tiles are disjoint, and
// every destination slot is still written by exactly one source node.
//
// ALIGNED (nx a multiple of 64, a row's node blocks under 2 GiB:
// phase_tb2_aligned): every row starts on a node-block boundary, so value i of
// column c in row v lies at the row's block base (uniform over the workgroup:
// scalar registers) plus the column's byte offset within the row's blocks
// (per lane, 32 bits, fixed for x, x - 1 and x + 1) plus i blocks of 64
// values, and no access needs per-lane 64-bit index arithmetic.  Other rows
// take the general node-block index.
// ---------------------------------------------------------------------------
constexpr int kTbMaxNx = 256;
constexpr int kTbHalo = 3;                          // overlap columns per side (TILED)
constexpr int kTbTileOut = kTbMaxNx - 2 * kTbHalo;  // stored columns per tile
#ifndef LBM_TB_SEG
#define LBM_TB_SEG 128
#endif
constexpr int kTbSeg = LBM_TB_SEG;  // rows per segment

// register state of one row of one column: h 0-8, low part of h_0, z 0-8, (phi u)
constexpr int kH = 0, kLO = 9, kZ = 10, kPU = 19, kNS = 21;

template <typename S, bool TILED, bool ALIGNED>
__global__ __launch_bounds__(kTbMaxNx) void k_phase_tb2(PhaseK k, const S* __restrict__ A,
                                                        S* __restrict__ B, int seg) {
    static_assert(TILED || ALIGNED, "whole rows are 64, 128, 192 or 256 columns");
    using C = S;
    constexpr bool RMASS = std::is_same<S, float>::value;
    using PL = PhasePlanes<S>;
    const int nx = k.nx, ny = k.ny;
    const int nseg = (ny + seg - 1) / seg;
    const int ntx = TILED ? (nx + kTbTileOut - 1) / kTbTileOut : 1;
    int w;
    if (!xcd_tile(ntx * nseg * k.batch, w)) return;  // whole workgroup, before any barrier
    const int tx = w % ntx;  // x-tile (TILED), x fastest
    w /= ntx;
    const int b = w / nseg;
    const int a = (w - b * nseg) * seg;
    const int e = min(a + seg, ny);
    const bool walls = k.bcy != 0;
    const int s1 = walls ? max(a - 2, 0) : a - 2;   // first row of step n
    const int e1 = walls ? min(e + 2, ny) : e + 2;  // end of step-n rows
    const int lastload = walls ? min(e1, ny - 1) : e1;
    const long long base = (long long)b * ny * nx;
    // x, xm, xp: the lane's column and its periodic neighbours in memory; lx,
    // lxm, lxp: the lane and its neighbour lanes in LDS (the same unless
    // TILED).
    const unsigned lx = threadIdx.x;
    unsigned x = lx;
    bool out = true;  // this lane stores its step-(n + 1) result
    if constexpr (TILED) {
        const int c = tx * kTbTileOut - kTbHalo + int(lx);
        x = unsigned(((c % nx) + nx) % nx);
        out = int(lx) >= kTbHalo && int(lx) < kTbMaxNx - kTbHalo && c < nx;
    }
    const unsigned xm = x == 0 ? nx - 1 : x - 1;
    const unsigned xp = x == unsigned(nx - 1) ? 0u : x + 1;
    const unsigned lxm = TILED ? (lx == 0 ? 0u : lx - 1) : xm;
    const unsigned lxp = TILED ? (lx == kTbMaxNx - 1 ? lx : lx + 1) : xp;

    __shared__ C phN[4][kTbMaxNx];   // phi_n, rows v mod 4
    __shared__ C phN1[4][kTbMaxNx];  // phi_{n+1}
    __shared__ C xch[12][kTbMaxNx];  // x-moving post-collision values of step n

    // memory row of virtual row v: virtual rows of a periodic segment lie in
    // [-3, ny + 2] and ny >= 4, so one correction wraps them
    auto rowoff = [&](int v) {
        const int r = v < 0 ? v + ny : (v >= ny ? v - ny : v);
        return base + (long long)r * nx;
    };
    // value i of the node in column slot c (0: x, 1: x - 1, 2: x + 1) of row v
    const unsigned xcol[3] = {x, xm, xp};
    unsigned boff[3];  // ALIGNED: byte offset of value 0 of those columns within a row
#pragma unroll
    for (int c = 0; c < 3; ++c)
        boff[c] = unsigned(((xcol[c] >> 6) * PL::NPL * kBlk + (xcol[c] & (kBlk - 1))) * sizeof(S));
    auto at = [&](auto* P, int v, int c, int i) {
        if constexpr (ALIGNED) {
            using B8 = std::conditional_t<std::is_const_v<std::remove_pointer_t<decltype(P)>>,
                                          const char, char>;
            auto* row = (B8*)P + (rowoff(v) >> 6) * (long long)(PL::NPL * kBlk * sizeof(S));
            return (decltype(P))(row + boff[c]) + i * kBlk;
        } else {
            return P + pidx<S>(i, rowoff(v) + xcol[c]);
        }
    };
    auto load_row = [&](int v, C (&s)[kNS]) {
#pragma unroll
        for (int i = 0; i < 9; ++i) s[kH + i] = C(*at(A, v, 0, PL::H + i));
#pragma unroll
        for (int i = 0; i < 9; ++i) s[kZ + i] = C(*at(A, v, 0, PL::Z + i));
        s[kLO] = RMASS ? C(*at(A, v, 0, PL::LO)) : C(0);
        s[kPU] = C(*at(A, v, 0, PL::PU));
        s[kPU + 1] = C(*at(A, v, 0, PL::PU + 1));
    };
    auto phi_of = [&](const C (&s)[kNS]) {
        const C hh[9] = {s[0], s[1], s[2], s[3], s[4], s[5], s[6], s[7], s[8]};
        return phi_sum(hh, s[kLO]);
    };
    // phi of row v into a ring, with the wall ghost rows (copies of the
    // first and last rows: zero normal gradient)
    auto put_phi = [&](C (&ring)[4][kTbMaxNx], int v, C ph) {
        ring[v & 3][lx] = ph;
        if (walls && v == 0) ring[3][lx] = ph;                // row -1
        if (walls && v == ny - 1) ring[ny & 3][lx] = ph;      // row ny
    };
    auto gather = [&](C (&ring)[4][kTbMaxNx], int v, C (&pn)[9]) {
        const C* rm = ring[(v - 1) & 3];
        const C* r0 = ring[v & 3];
        const C* rp = ring[(v + 1) & 3];
        pn[0] = r0[lx];
        pn[1] = r0[lxp];
        pn[2] = rp[lx];
        pn[3] = r0[lxm];
        pn[4] = rm[lx];
        pn[5] = rp[lxp];
        pn[6] = rp[lxm];
        pn[7] = rm[lxm];
        pn[8] = rm[lxp];
    };

    // Register slots: slot (u - s1) mod 5 holds row u of
    //   Ld: the stored state (rows v and v + 1 are live),
    //   Ac: the accumulated step-(n+1) state (rows v - 3 .. v + 1).
    // The row loop is unrolled five times, so every slot index is a
    // compile-time constant and no row is copied between registers.
    C Ld[5][kNS], Ac[5][kNS];
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
        for (int q = 0; q < kNS; ++q) Ld[j][q] = Ac[j][q] = C(0);
    // prologue: phi_n of rows s1 - 1 and s1, state of row s1 (slot 0)
    if (!walls || s1 > 0) {
        load_row(s1 - 1, Ld[4]);
        put_phi(phN, s1 - 1, phi_of(Ld[4]));
    }
    load_row(s1, Ld[0]);
    put_phi(phN, s1, phi_of(Ld[0]));
    // (the first barrier of the row step orders these LDS writes)

    // one row step at row v, v - s1 = J (mod 5)
    auto row_step = [&](int v, auto Jc) {
        constexpr int J = decltype(Jc)::value;
        constexpr int s0 = J % 5, sn = (J + 1) % 5;          // rows v, v + 1
        constexpr int sm1 = (J + 4) % 5, sm3 = (J + 2) % 5;  // rows v - 1, v - 3
        const bool do_n = v < e1;
        const bool do_load = v + 1 <= lastload;
        const int r = v - 3;
        // the load is unconditional (the last rows re-read an in-bounds row),
        // so the compiler can see that every slot is overwritten before it
        // is read and keeps only the live rows in registers
        load_row(do_load ? v + 1 : lastload, Ld[sn]);
        __syncthreads();  // phi_{n+1} of row v - 2 and the previous exchange reads are done
        // ---- step n + 1 at row r = v - 3, straight to memory
        if (r >= a && r < e && out) {
            C pn[9], h[9], z[9], hs[9], zst[9], pux, puy;
            S h0hi, h0lo;
            gather(phN1, r, pn);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                h[i] = Ac[sm3][kH + i];
                z[i] = Ac[sm3][kZ + i];
            }
            const PhaseLocal<C> L = phase_local(k, pn, z);
            phase_collide<S, C>(k, L, h, Ac[sm3][kLO], z, Ac[sm3][kPU], Ac[sm3][kPU + 1], hs, h0hi,
                                h0lo, zst, pux, puy);
            st(at(B, r, 0, PL::PU), S(pux));
            st(at(B, r, 0, PL::PU + 1), S(puy));
            st(at(B, r, 0, PL::H), h0hi);
            if constexpr (RMASS) st(at(B, r, 0, PL::LO), h0lo);
            st(at(B, r, 0, PL::Z), S(zst[0]));
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const int ryd = r + EY[i];
                if (walls && (ryd < 0 || ryd >= ny)) {
                    st(at(B, r, 0, PL::H + OPP[i]), S(hs[i]));
                    st(at(B, r, 0, PL::Z + OPP[i]), S(zst[i]));
                } else {
                    const int c = EX[i] == 0 ? 0 : (EX[i] > 0 ? 2 : 1);
                    st(at(B, ryd, c, PL::H + i), S(hs[i]));
                    st(at(B, ryd, c, PL::Z + i), S(zst[i]));
                }
            }
        }
        // ---- phi_n of row v + 1
        if (do_load) put_phi(phN, v + 1, phi_of(Ld[sn]));
        __syncthreads();
        // ---- step n at row v
        C hs[9], zst[9], pux = C(0), puy = C(0);
        S h0hi = S(0), h0lo = S(0);
        if (do_n) {
            C pn[9], h[9], z[9];
            gather(phN, v, pn);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                h[i] = Ld[s0][kH + i];
                z[i] = Ld[s0][kZ + i];
            }
            const PhaseLocal<C> L = phase_local(k, pn, z);
            phase_collide<S, C>(k, L, h, Ld[s0][kLO], z, Ld[s0][kPU], Ld[s0][kPU + 1], hs, h0hi,
                                h0lo, zst, pux, puy);
            xch[0][lx] = hs[1];
            xch[1][lx] = hs[3];
            xch[2][lx] = hs[5];
            xch[3][lx] = hs[6];
            xch[4][lx] = hs[7];
            xch[5][lx] = hs[8];
            xch[6][lx] = zst[1];
            xch[7][lx] = zst[3];
            xch[8][lx] = zst[5];
            xch[9][lx] = zst[6];
            xch[10][lx] = zst[7];
            xch[11][lx] = zst[8];
        }
        __syncthreads();
        if (do_n) {
            // pushes of row v: +y movers to row v + 1, rest and x movers to
            // row v, -y movers to row v - 1 (x movers come from x -+ 1)
            C(&A0)[kNS] = Ac[s0];
            C(&Ap)[kNS] = Ac[sn];
            C(&A1)[kNS] = Ac[sm1];
            A0[kH + 0] = C(h0hi);
            A0[kLO] = C(h0lo);
            A0[kZ + 0] = zst[0];
            A0[kPU] = pux;
            A0[kPU + 1] = puy;
            A0[kH + 1] = xch[0][lxm];
            A0[kH + 3] = xch[1][lxp];
            A0[kZ + 1] = xch[6][lxm];
            A0[kZ + 3] = xch[7][lxp];
            // +y movers to row v + 1, -y movers to row v - 1.  Written
            // unconditionally (branch-free, so every slot stays in registers):
            // at a wall the row beyond it does not exist and its slot is
            // overwritten before it is read again.
            Ap[kH + 2] = hs[2];
            Ap[kH + 5] = xch[2][lxm];
            Ap[kH + 6] = xch[3][lxp];
            Ap[kZ + 2] = zst[2];
            Ap[kZ + 5] = xch[8][lxm];
            Ap[kZ + 6] = xch[9][lxp];
            A1[kH + 4] = hs[4];
            A1[kH + 7] = xch[4][lxp];
            A1[kH + 8] = xch[5][lxm];
            A1[kZ + 4] = zst[4];
            A1[kZ + 7] = xch[10][lxp];
            A1[kZ + 8] = xch[11][lxm];
            // top wall: the +y movers come back reversed into the node's -y
            // slots (below the top row, the next row's pushes overwrite them)
            A0[kH + 4] = hs[2];
            A0[kH + 7] = hs[5];
            A0[kH + 8] = hs[6];
            A0[kZ + 4] = zst[2];
            A0[kZ + 7] = zst[5];
            A0[kZ + 8] = zst[6];
            // bottom wall: the -y movers come back reversed into the +y slots
            // (elsewhere those hold the pushes of the row below)
            const bool bottom = walls && v == 0;
            A0[kH + 2] = bottom ? hs[4] : A0[kH + 2];
            A0[kH + 5] = bottom ? hs[7] : A0[kH + 5];
            A0[kH + 6] = bottom ? hs[8] : A0[kH + 6];
            A0[kZ + 2] = bottom ? zst[4] : A0[kZ + 2];
            A0[kZ + 5] = bottom ? zst[7] : A0[kZ + 5];
            A0[kZ + 6] = bottom ? zst[8] : A0[kZ + 6];
        }
        // ---- phi_{n+1} of row v - 1, whose state is complete now
        {
            const int q = v - 1;
            const bool need = q >= a - 1 && q <= e && (!walls || (q >= 0 && q < ny));
            if (need) put_phi(phN1, q, phi_of(Ac[sm1]));
        }
    };
    const int vend = e + 3;
    for (int v = s1; v < vend; v += 5) {
        row_step(v, std::integral_constant<int, 0>{});
        if (v + 1 >= vend) break;
        row_step(v + 1, std::integral_constant<int, 1>{});
        if (v + 2 >= vend) break;
        row_step(v + 2, std::integral_constant<int, 2>{});
        if (v + 3 >= vend) break;
        row_step(v + 3, std::integral_constant<int, 3>{});
        if (v + 4 >= vend) break;
        row_step(v + 4, std::integral_constant<int, 4>{});
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
__global__ void k_chan_init(ChanK k, const double* __restrict__ fld, S* __restrict__ A) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    const long long P = k.P;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        const double rho = fld[n], ux = fld[P + n] / k.c, uy = fld[2 * P + n] / k.c;
        const double th = fld[3 * P + n] - k.T_ref;
        const double uu = ux * ux + uy * uy;
        for (int i = 0; i < 9; ++i) {
            const double eu = EX[i] * ux + EY[i] * uy;
            A[bidx(k.npl, i, n)] = S(wgt<double>(i) * ((rho - k.rho_ref) +
                                                       rho * (3 * eu + 4.5 * eu * eu - 1.5 * uu)));
        }
        if (k.thermal && k.tq == 9)
            for (int i = 0; i < 9; ++i)
                A[bidx(k.npl, 9 + i, n)] =
                    S(wgt<double>(i) * th * (1 + 3 * (EX[i] * ux + EY[i] * uy)));
        else if (k.thermal)
            for (int i = 0; i < 5; ++i)
                A[bidx(k.npl, 9 + i, n)] =
                    S(wgt5<double>(i) * th * (1 + 3 * (EX5[i] * ux + EY5[i] * uy)));
    }
}

template <typename S>
__global__ void k_phase_init(PhaseK k, const double* __restrict__ fld, S* __restrict__ A) {
    constexpr bool RMASS = std::is_same<S, float>::value;
    using PL = PhasePlanes<S>;
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
            A[pidx<S>(PL::H + i, n)] = hv;
            hsum += double(hv);
        }
        const double h0 = phi - hsum;  // rest population closes the node's phi exactly
        const S hi = S(h0);
        A[pidx<S>(PL::H, n)] = hi;
        if (RMASS) A[pidx<S>(PL::LO, n)] = S(h0 - double(hi));
        for (int i = 0; i < 9; ++i) {
            const double eu = EX[i] * ux + EY[i] * uy;
            const double w = wgt<double>(i);
            A[pidx<S>(PL::Z + i, n)] =
                S(ph * (i == 0 ? w - 1 : w) + rho * w * (3 * eu + 4.5 * eu * eu - 1.5 * uu));
        }
        A[pidx<S>(PL::PU, n)] = S(phi * ux);
        A[pidx<S>(PL::PU + 1, n)] = S(phi * uy);
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
__global__ void k_chan_macros(ChanK k, const S* __restrict__ A, double* __restrict__ out) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    const long long P = k.P;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        double th = 0.0;
        if (k.thermal) {
            double s = 0;
            for (int i = 0; i < k.tq; ++i) s += double(A[bidx(k.npl, 9 + i, n)]);
            th = s + 0.5 * k.qdt;
        }
        double fx, fy;
        chan_force(k, th, fx, fy);
        double d[9], drho, rho, ux, uy;
        chan_flow_macros<double, S>(A, k.npl, n, k.rho_ref, fx, fy, d, drho, rho, ux, uy);
        out[n] = rho;
        out[2 * P + n] = ux * k.c;
        out[3 * P + n] = uy * k.c;
        out[4 * P + n] = k.T_ref + th;
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
                                                 D3K d3, P3K p3, const S* __restrict__ pops,
                                                 int npop, double* __restrict__ partial) {
    const int b = blockIdx.y;
    long long M, P;
    if (lattice == LBM_D2Q9_PHASE) { M = (long long)pk.nx * pk.ny; P = pk.P; }
    else if (lattice == LBM_D2Q9_D2Q5) { M = (long long)ck.nx * ck.ny; P = ck.P; }
    else if (lattice == LBM_D3Q19) { M = (long long)d3.nx * d3.ny * d3.nz; P = d3.P; }
    else if (lattice == LBM_D3Q19_PHASE) { M = (long long)p3.nx * p3.ny * p3.nz; P = p3.P; }
    else { M = dk.n; P = dk.n; }
    const long long base = b * M;
    double v[4] = {0, 0, 0, 0};
    for (long long j = blockIdx.x * 256LL + threadIdx.x; j < M; j += 256LL * gridDim.x) {
        const long long n = base + j;
        // value i of node n: node blocks for the 2D and 3D lattices, planes
        // of stride P for the 1D ones
        auto at = [&](int i) {
            constexpr int npl3 = std::is_same<S, float>::value ? 42 : 41;
            const long long j = lattice == LBM_D2Q9_PHASE    ? pidx<S>(i, n)
                                : lattice == LBM_D2Q9_D2Q5   ? bidx(ck.npl, i, n)
                                : lattice == LBM_D3Q19       ? bidx(19, i, n)
                                : lattice == LBM_D3Q19_PHASE ? bidx(npl3, i, n)
                                                             : i * P + n;
            return double(pops[j]);
        };
        double cnt = 0;
        for (int i = 0; i < npop; ++i)
            if (!isfinite(at(i))) cnt += 1;
        v[3] += cnt;
        if (lattice == LBM_D2Q9_PHASE) {
            double a = 0;
            for (int i = 0; i < 9; ++i) a += at(PhasePlanes<S>::H + i);
            if (std::is_same<S, float>::value) a += at(PhasePlanes<S>::LO);
            v[1] += a;
            v[0] += pk.rho_g + a * (pk.rho_l - pk.rho_g);
        } else if (lattice == LBM_D3Q19_PHASE) {
            double a = 0;
            for (int i = 0; i < 19; ++i) a += at(i);
            if (std::is_same<S, float>::value) a += at(38);
            v[1] += a;
            v[0] += p3.rho_g + a * (p3.rho_l - p3.rho_g);
        } else if (lattice == LBM_D3Q19) {
            double a = 0;
            for (int i = 0; i < 19; ++i) a += at(i);
            v[0] += d3.rho_ref + a;
        } else if (lattice == LBM_D2Q9_D2Q5) {
            double a = 0;
            for (int i = 0; i < 9; ++i) a += at(i);
            v[0] += ck.rho_ref + a;
            if (ck.thermal) {
                double s = 0;
                for (int i = 0; i < ck.tq; ++i) s += at(9 + i);
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

// Non-finite watch: every node value of planes [0, nplanes) (N nodes; plane
// stride P, or the node-block layout of nplanes planes when blocked) that is
// NaN or infinite lowers *first to t.  Grid (blocks, planes).
template <typename S>
__global__ __launch_bounds__(256) void k_nonfinite_watch(const S* __restrict__ pops, long long P,
                                                         long long N, int blocked,
                                                         unsigned long long t,
                                                         unsigned long long* __restrict__ first) {
    const int i = blockIdx.y;
    bool bad = false;
    for (long long n = blockIdx.x * 256LL + threadIdx.x; n < N; n += 256LL * gridDim.x)
        bad |= !isfinite(pops[blocked ? bidx(gridDim.y, i, n) : i * P + n]);
    if (bad) atomicMin(first, t);
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
__global__ void k_nusselt(ChanK k, const S* __restrict__ A, const S* __restrict__ qw,
                          double qsi, double Dh, double kc, double dx,
                          double* __restrict__ Tb, double* __restrict__ Tw,
                          double* __restrict__ Nu) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= k.nx) return;
    double su = 0, suT = 0, T0 = 0, T1 = 0;
    for (int y = 0; y < k.ny; ++y) {
        const long long n = (long long)y * k.nx + x;
        double s = 0;
        for (int i = 0; i < k.tq; ++i) s += double(A[bidx(k.npl, 9 + i, n)]);
        const double T = k.T_ref + s + 0.5 * k.qdt;
        double fx, fy;
        chan_force(k, T - k.T_ref, fx, fy);
        double d[9], drho, rho, ux, uy;
        chan_flow_macros<double, S>(A, k.npl, n, k.rho_ref, fx, fy, d, drho, rho, ux, uy);
        su += ux;
        suT += ux * T;
        if (y == 0) T0 = T;
        if (y == k.ny - 1) T1 = T;
    }
    const double q = double(qw[x]) * qsi;  // W/m^2 including the time modulation
    const double tb = suT / su;
    // wall temperature: mean of the two wall-adjacent nodes, or the lower one
    // with a symmetry plane on top; plus the half-cell conduction q dx / 2k
    const double tw = (k.bcy == 2 ? T0 : 0.5 * (T0 + T1)) + q * dx / (2.0 * kc);
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
// The channel step runs on one-row tiles (64 x 1, one wave per workgroup) at
// every size.  On the paper-sized channels they spread the grid over more CUs
// than 64 x 4 tiles (C2's 800 x 40 under graph replay 5.37 -> 5.15 us per
// step, C5's 1600 x 80 6.37 -> 6.23 us; two-row tiles 5.27 and 6.15), and on
// the 16384 x 2048 grid the step takes 0.715-0.723 ms against 0.728-0.737 ms
// with 64 x 4 tiles (64 x 2: 0.715-0.722; 64 x 8: 0.771; 64 x 4 capped at
// four or three workgroups per CU by an LDS reserve: 0.793 and 1.236 ms).
// An LDS reserve per one-wave workgroup caps the waves resident per CU: 26
// in FP32 (the register count alone allows 32), 12 in FP64 (20).  With more
// waves, more population streams are open in DRAM at once; on the 16384 x
// 2048 grid: FP32 0.700 ms per step uncapped, 0.666 ms at 26 or 30 waves,
// 0.671 at 22 or 24, 0.699 at 20, 0.737 at 16; FP64 1.420 ms uncapped,
// 1.349 at 16, 1.318 at 12, 1.360 at 10, 1.429 at 8.  The paper-sized grids
// (launch-bound) are unchanged.
constexpr unsigned kChanLdsReserve32 = 6144, kChanLdsReserve64 = 13312;
template <typename S>
hipError_t launch_chan_step(const ChanK& k, const S* a, S* b, const S* qw, const S* uin,
                            const S* tin, double mod, hipStream_t s) {
    const long long tiles = (long long)((k.nx + 63) / 64) * k.ny * k.batch;
    dim3 blk(64), grd(unsigned((tiles + kXCD - 1) / kXCD * kXCD));
    const unsigned lds = sizeof(S) == 4 ? kChanLdsReserve32 : kChanLdsReserve64;
    if (k.tq == 9)
        hipLaunchKernelGGL((k_chan_step<S, 9>), grd, blk, lds, s, k, a, b, qw, uin, tin, S(mod));
    else
        hipLaunchKernelGGL((k_chan_step<S, 5>), grd, blk, lds, s, k, a, b, qw, uin, tin, S(mod));
    return hipGetLastError();
}

// The two-step channel kernel covers flow with temperature (D2Q5 or the D2Q9
// set, with or without the Boussinesq force), every x and y boundary of the
// channel lattice, and at least two columns and rows.
bool chan_tb2_fits(const ChanK& k) {
    return k.flow && k.thermal && (k.tq == 5 || k.tq == 9) && k.npl == ct_nv(k.tq) &&
           k.bcx >= 0 && k.bcx <= 2 && k.bcy >= 0 && k.bcy <= 2 && k.nx >= 2 && k.ny >= 2;
}
int chan_tb2_ntx(const ChanK& k) { return (k.nx + kCtOut - 1) / kCtOut; }
// Share of the launched lanes whose columns are stored.
double chan_tb2_lane_use(const ChanK& k) {
    return double(k.nx) / (double(chan_tb2_ntx(k)) * kCtLanes);
}
template <typename S>
bool chan_tb2_aligned(const ChanK& k) {
    return k.nx % kBlk == 0 && (long long)k.nx * ct_nv(k.tq) * (long long)sizeof(S) < (1LL << 31);
}
long long chan_tb2_workgroups(const ChanK& k, int seg) {
    return (long long)((k.ny + seg - 1) / seg) * k.batch * chan_tb2_ntx(k);
}

// Rows per segment, by the launch-round model of the two-phase kernel: a
// workgroup marches seg + 2 rows (its segment, one row of overlap below and
// one of lag above), the GPU holds `slots` workgroups at once, and the
// segment length (at least 32 rows, or the whole replica) minimises
// ceil(workgroups / slots) (seg + 2).  On the 16384 x 2048 channel (66
// x-tiles, three workgroups per CU) it picks 90 rows, the fastest of 32 to
// 512 rows in a sweep (0.420 ms per step; 187 rows 0.427, 64 rows 0.434,
// 128 rows 0.541, 256 rows 0.525).
// The instance of the two-step channel kernel for a configuration.
template <typename S>
auto chan_tb2_kernel(const ChanK& k) {
    const bool ends = k.bcx == 2 || k.bcy == 2;
    if (k.tq == 9) {
        if (chan_tb2_aligned<S>(k))
            return ends ? k_chan_tb2<S, true, true, 9> : k_chan_tb2<S, true, false, 9>;
        return ends ? k_chan_tb2<S, false, true, 9> : k_chan_tb2<S, false, false, 9>;
    }
    if (chan_tb2_aligned<S>(k))
        return ends ? k_chan_tb2<S, true, true, 5> : k_chan_tb2<S, true, false, 5>;
    return ends ? k_chan_tb2<S, false, true, 5> : k_chan_tb2<S, false, false, 5>;
}

template <typename S>
int chan_tb2_seg(const ChanK& k) {
    const int ny = k.ny;
    int dev = 0, cus = 0, per_cu = 0;
    long long slots = 1024;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, chan_tb2_kernel<S>(k), kCtLanes, 0) ==
            hipSuccess &&
        cus > 0 && per_cu > 0)
        slots = (long long)cus * per_cu;
    const long long units = (long long)k.batch * chan_tb2_ntx(k);
    const int lo = ny < 32 ? ny : 32;
    int best = ny;
    long long best_cost = -1;
    for (int seg = ny; seg >= lo; --seg) {
        const long long nseg = (ny + seg - 1) / seg;
        if (seg < ny && seg - 1 >= lo && (ny + seg - 2) / (seg - 1) == nseg)
            continue;  // a shorter segment gives the same count: take the shortest of them
        const long long rounds = (units * nseg + slots - 1) / slots;
        const long long cost = rounds * (seg + 2);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = seg;
        }
    }
    return best;
}

template <typename S>
hipError_t launch_chan_tb2(const ChanK& k, const S* a, S* b, const S* qw, const S* uin,
                           const S* tin, double mod0, double mod1, int seg, hipStream_t s) {
    if (!chan_tb2_fits(k) || seg < 1) return hipErrorInvalidValue;
    const long long wgs = chan_tb2_workgroups(k, seg);
    if ((wgs + kXCD - 1) / kXCD * kXCD > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grd(unsigned((wgs + kXCD - 1) / kXCD * kXCD)), blk(kCtLanes);
    hipLaunchKernelGGL(chan_tb2_kernel<S>(k), grd, blk, 0, s, k, a, b, qw, uin, tin, S(mod0),
                       S(mod1), seg);
    return hipGetLastError();
}

// FP32 steps run on 256-node tiles, four resident per CU (kPhaseLdsReserve).
// Measured against 512-node tiles (two per CU): equal on 1024 replicas of
// 256^2, faster on smaller grids (64 replicas 146 -> 141 us per step, C4's
// 4 x 512 replica under graph replay 5.22 -> 4.61 us).  FP64 steps and the
// macro evaluation keep 512-node tiles (FP64: 4 % slower on 256-node tiles).

// One launch of k_phase with the tile shape for the replica width: 64 x TY,
// or, for nx in {4, 8, 16, 32}, nx x (512 / nx); half as many rows for FP32
// steps.
template <typename S, typename C, bool MACROS>
hipError_t launch_phase_kernel(const PhaseK& k, const S* a, S* b, double* out, unsigned lds,
                               hipStream_t s) {
    auto ntiles = [&](int tx, int ty) {
        return (long long)((k.nx + tx - 1) / tx) * ((k.ny + ty - 1) / ty) * k.batch;
    };
    const bool half = !MACROS && std::is_same<S, float>::value;
    auto go = [&](auto kern, int tx, int ty) {
        const long long tiles = ntiles(tx, ty);
        dim3 blk(tx, ty), grd(unsigned((tiles + kXCD - 1) / kXCD * kXCD));
        hipLaunchKernelGGL(kern, grd, blk, lds, s, k, a, b, out);
        return hipGetLastError();
    };
    if (half) {
        switch (k.nx) {
            case 4: return go(k_phase<S, C, MACROS, 4, 64>, 4, 64);
            case 8: return go(k_phase<S, C, MACROS, 8, 32>, 8, 32);
            case 16: return go(k_phase<S, C, MACROS, 16, 16>, 16, 16);
            case 32: return go(k_phase<S, C, MACROS, 32, 8>, 32, 8);
            default: return go(k_phase<S, C, MACROS, TX, TY / 2>, TX, TY / 2);
        }
    }
    switch (k.nx) {
        case 4: return go(k_phase<S, C, MACROS, 4, 128>, 4, 128);
        case 8: return go(k_phase<S, C, MACROS, 8, 64>, 8, 64);
        case 16: return go(k_phase<S, C, MACROS, 16, 32>, 16, 32);
        case 32: return go(k_phase<S, C, MACROS, 32, 16>, 32, 16);
        default: return go(k_phase<S, C, MACROS>, TX, TY);
    }
}

#ifndef LBM_PERSIST_MIN_THREADS
#define LBM_PERSIST_MIN_THREADS 128
#endif

// Tile shape of the many-steps kernel for a workgroup of `threads` threads:
// nx x threads/nx for the narrow replicas (nx = 4, 8, 16, 32), else 64 x
// threads/64 (at least 256 threads, so that a thread holds each ring node).
void persist_shape(const PhaseK& k, int threads, int* tx, int* ty) {
    const bool narrow = k.nx == 4 || k.nx == 8 || k.nx == 16 || k.nx == 32;
    if (!narrow && threads < 256) threads = 256;
    *tx = narrow ? k.nx : 64;
    *ty = threads / *tx;
}

long long persist_tiles(const PhaseK& k, int threads) {
    int tx, ty;
    persist_shape(k, threads, &tx, &ty);
    return (long long)((k.nx + tx - 1) / tx) * ((k.ny + ty - 1) / ty) * k.batch;
}

// At most kPersistMaxTiles tiles; with a one-node tail every tile of a
// replica is watched by one wave, so a replica then has at most 64.
bool persist_ok(const PhaseK& k, int threads) {
    int tx, ty;
    persist_shape(k, threads, &tx, &ty);
    const int gx = (k.nx + tx - 1) / tx, gy = (k.ny + ty - 1) / ty;
    const bool thin = (gx > 1 && k.nx - (gx - 1) * tx < 2) || (gy > 1 && k.ny - (gy - 1) * ty < 2);
    return persist_tiles(k, threads) <= kPersistMaxTiles && !(thin && (long long)gx * gy > 64);
}

// The smallest workgroup (most tiles, least work per CU) that fits; 0 if
// none does.
int persist_threads(const PhaseK& k) {
    for (int t = LBM_PERSIST_MIN_THREADS; t <= 512; t *= 2)
        if (persist_ok(k, t)) return t;
    return 0;
}

bool phase_persist_fits(const PhaseK& k) { return persist_threads(k) != 0; }

template <typename S>
hipError_t launch_phase_persist(const PhaseK& k, S* A, S* B, int nsteps, unsigned epoch0,
                                unsigned* flags, unsigned* err, bool arith64, hipStream_t s) {
    if (arith64 && !std::is_same<S, float>::value) return hipErrorInvalidValue;
    const int threads = persist_threads(k);
    if (!threads || nsteps < 1) return hipErrorInvalidValue;
    int tx, ty;
    persist_shape(k, threads, &tx, &ty);
    const unsigned tiles = unsigned(persist_tiles(k, threads));
    void* args[] = {(void*)&k, (void*)&A, (void*)&B, (void*)&nsteps, (void*)&epoch0, (void*)&flags,
                    (void*)&err};
    auto go = [&](const void* kern) {
        return hipLaunchCooperativeKernel(kern, dim3(tiles), dim3(tx, ty), args, 0, s);
    };
#define LBM_PERSIST_CASE(X, Y)                                                                 \
    if (tx == X && ty == Y)                                                                    \
        return go(arith64 ? reinterpret_cast<const void*>(&k_phase_persist<S, double, X, Y>)   \
                          : reinterpret_cast<const void*>(&k_phase_persist<S, S, X, Y>));
    LBM_PERSIST_CASE(4, 32) LBM_PERSIST_CASE(4, 64) LBM_PERSIST_CASE(4, 128)
    LBM_PERSIST_CASE(8, 16) LBM_PERSIST_CASE(8, 32) LBM_PERSIST_CASE(8, 64)
    LBM_PERSIST_CASE(16, 8) LBM_PERSIST_CASE(16, 16) LBM_PERSIST_CASE(16, 32)
    LBM_PERSIST_CASE(32, 4) LBM_PERSIST_CASE(32, 8) LBM_PERSIST_CASE(32, 16)
    LBM_PERSIST_CASE(64, 4) LBM_PERSIST_CASE(64, 8)
#undef LBM_PERSIST_CASE
    return hipErrorInvalidValue;
}

template <typename S>
hipError_t launch_phase_step(const PhaseK& k, const S* a, S* b, bool arith64, hipStream_t s) {
    const unsigned lds = std::is_same<S, float>::value ? kPhaseLdsReserve : 0u;  // half tiles
    if (arith64) {  // FP32 storage, every step evaluated in FP64
        if (!std::is_same<S, float>::value) return hipErrorInvalidValue;
        return launch_phase_kernel<S, double, false>(k, a, b, (double*)nullptr, lds, s);
    }
    return launch_phase_kernel<S, S, false>(k, a, b, (double*)nullptr, lds, s);
}

// The two-step kernel takes a whole row per workgroup when nx is a multiple
// of 64 up to 256, and x-tiles of kTbTileOut stored columns otherwise; y
// needs at least 4 rows (virtual rows wrap with one correction).
bool phase_tb2_fits(const PhaseK& k) { return k.ny >= 4 && k.nx >= 1; }
bool phase_tb2_tiled(const PhaseK& k) { return !(k.nx % 64 == 0 && k.nx <= kTbMaxNx); }
int phase_tb2_ntx(const PhaseK& k) {
    return phase_tb2_tiled(k) ? (k.nx + kTbTileOut - 1) / kTbTileOut : 1;
}
// Share of the launched lanes whose columns are stored (1 for whole rows).
double phase_tb2_lane_use(const PhaseK& k) {
    return phase_tb2_tiled(k) ? double(k.nx) / (double(phase_tb2_ntx(k)) * kTbMaxNx) : 1.0;
}

// Whether the two-step kernel addresses rows through a scalar block base and
// 32-bit lane offsets: nx a multiple of 64, and the byte offset of the last
// column within a row's node blocks (nx values per state value) below 2^31.
template <typename S>
bool phase_tb2_aligned(const PhaseK& k) {
    return k.nx % kBlk == 0 &&
           (long long)k.nx * PhasePlanes<S>::NPL * (long long)sizeof(S) < (1LL << 31);
}

// Rows per segment.  Every workgroup marches seg + 5 rows (its segment, two
// rows of overlap below and three of lag above), all workgroups take the
// same time, and the GPU holds `slots` of them at once, so a launch costs
// about ceil(workgroups / slots) (seg + 5) row steps.  The segment length
// (at least 64 rows, or the whole replica) minimises that, preferring longer
// segments on ties: 1024 replicas of 256^2 in FP32 (512 slots) keep whole
// replicas (two full rounds); the 8192^2 domain in 33 x-tiles takes 265-row
// segments (1023 workgroups, two rounds) instead of 128-row ones (2112
// workgroups: a fifth, nearly empty round).
template <typename S>
int phase_tb2_seg(const PhaseK& k) {
    const int ny = k.ny;
    int dev = 0, cus = 0, per_cu = 0;
    const bool tiled = phase_tb2_tiled(k);
    long long slots = 512;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        (tiled ? (phase_tb2_aligned<S>(k)
                      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &per_cu, k_phase_tb2<S, true, true>, kTbMaxNx, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &per_cu, k_phase_tb2<S, true, false>, kTbMaxNx, 0))
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_phase_tb2<S, false, true>,
                                                              k.nx, 0)) == hipSuccess &&
        cus > 0 && per_cu > 0)
        slots = (long long)cus * per_cu;
    const long long units = (long long)k.batch * phase_tb2_ntx(k);
    const int lo = ny < kTbSeg ? ny : kTbSeg / 2;
    int best = ny;
    long long best_cost = -1;
    for (int seg = ny; seg >= lo; --seg) {
        const long long nseg = (ny + seg - 1) / seg;
        if (seg < ny && (ny + seg - 2) / (seg - 1 > 0 ? seg - 1 : 1) == nseg && seg - 1 >= lo)
            continue;  // a shorter segment gives the same count: take the shortest of them
        const long long rounds = (units * nseg + slots - 1) / slots;
        const long long cost = rounds * (seg + 5);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = seg;
        }
    }
    return best;
}

long long phase_tb2_workgroups(const PhaseK& k, int seg) {
    return (long long)((k.ny + seg - 1) / seg) * k.batch * phase_tb2_ntx(k);
}

template <typename S>
hipError_t launch_phase_tb2(const PhaseK& k, const S* a, S* b, int seg, hipStream_t s) {
    if (!phase_tb2_fits(k) || seg < 1) return hipErrorInvalidValue;
    const long long wgs = phase_tb2_workgroups(k, seg);
    if ((wgs + kXCD - 1) / kXCD * kXCD > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grd(unsigned((wgs + kXCD - 1) / kXCD * kXCD));
    if (!phase_tb2_tiled(k))
        hipLaunchKernelGGL((k_phase_tb2<S, false, true>), grd, dim3(k.nx), 0, s, k, a, b, seg);
    else if (phase_tb2_aligned<S>(k))
        hipLaunchKernelGGL((k_phase_tb2<S, true, true>), grd, dim3(kTbMaxNx), 0, s, k, a, b, seg);
    else
        hipLaunchKernelGGL((k_phase_tb2<S, true, false>), grd, dim3(kTbMaxNx), 0, s, k, a, b, seg);
    return hipGetLastError();
}

hipError_t launch_d1(const D1K& k, double* g, int nsteps, hipStream_t s) {
    hipLaunchKernelGGL(k_d1, dim3(1), dim3(1024), 0, s, k, g, nsteps);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_chan_init(const ChanK& k, const double* fields, S* a, hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    hipLaunchKernelGGL(k_chan_init<S>, dim3(grid1(N, 256)), dim3(256), 0, s, k, fields, a);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_phase_init(const PhaseK& k, const double* fields, S* a, hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    hipLaunchKernelGGL(k_phase_init<S>, dim3(grid1(N, 256)), dim3(256), 0, s, k, fields, a);
    return hipGetLastError();
}

hipError_t launch_d1_init(const D1K& k, const double* T, double* g, hipStream_t s) {
    hipLaunchKernelGGL(k_d1_init, dim3((k.n + 255) / 256), dim3(256), 0, s, k, T, g);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_chan_macros(const ChanK& k, const S* a, double* out, hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny;
    hipLaunchKernelGGL(k_chan_macros<S>, dim3(grid1(N, 256)), dim3(256), 0, s, k, a, out);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_phase_macros(const PhaseK& k, const S* a, double* out, hipStream_t s) {
    return launch_phase_kernel<S, double, true>(k, a, (S*)nullptr, out, 0u, s);
}

hipError_t launch_d1_macros(const D1K& k, const double* g, double* out, long long P,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_d1_macros, dim3((k.n + 255) / 256), dim3(256), 0, s, k, g, out, P);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_reduce(int lattice, const ChanK& ck, const PhaseK& pk, const D1K& dk,
                         const D3K& d3, const P3K& p3, const S* pops, int npop, double* partial,
                         double* out, hipStream_t s) {
    const int batch = lattice == LBM_D2Q9_PHASE    ? pk.batch
                      : lattice == LBM_D2Q9_D2Q5    ? ck.batch
                      : lattice == LBM_D3Q19        ? d3.batch
                      : lattice == LBM_D3Q19_PHASE  ? p3.batch
                                                    : 1;
    hipLaunchKernelGGL(k_reduce1<S>, dim3(kRedBlocks, batch), dim3(256), 0, s, lattice, ck, pk,
                       dk, d3, p3, pops, npop, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce2, dim3((batch * 4 + 63) / 64), dim3(64), 0, s, partial, out,
                       batch);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_nonfinite_watch(const S* pops, long long P, long long N, int nplanes,
                                  bool blocked, unsigned long long t, unsigned long long* first,
                                  hipStream_t s) {
    const long long blocks = std::min<long long>((N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_nonfinite_watch<S>, dim3(unsigned(blocks), nplanes), dim3(256), 0, s,
                       pops, P, N, int(blocked), t, first);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_nusselt(const ChanK& k, const S* a, const S* qw, double qsi, double Dh,
                          double kc, double dx, int x_dev, double* Tb, double* Tw, double* Nu,
                          double* small, hipStream_t s) {
    hipLaunchKernelGGL(k_nusselt<S>, dim3((k.nx + 255) / 256), dim3(256), 0, s, k, a, qw, qsi,
                       Dh, kc, dx, Tb, Tw, Nu);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nusselt_mean, dim3(1), dim3(64), 0, s, Nu, Tb, k.nx, x_dev, small);
    return hipGetLastError();
}

#define LBM_INST(S)                                                                              \
    template hipError_t launch_chan_step<S>(const ChanK&, const S*, S*, const S*, const S*,     \
                                            const S*, double, hipStream_t);                       \
    template hipError_t launch_phase_step<S>(const PhaseK&, const S*, S*, bool, hipStream_t);    \
    template hipError_t launch_phase_tb2<S>(const PhaseK&, const S*, S*, int, hipStream_t);      \
    template hipError_t launch_chan_tb2<S>(const ChanK&, const S*, S*, const S*, const S*,      \
                                           const S*, double, double, int, hipStream_t);           \
    template int chan_tb2_seg<S>(const ChanK&);                                                  \
    template int phase_tb2_seg<S>(const PhaseK&);                                                \
    template hipError_t launch_phase_persist<S>(const PhaseK&, S*, S*, int, unsigned, unsigned*,  \
                                                unsigned*, bool, hipStream_t);                    \
    template hipError_t launch_chan_init<S>(const ChanK&, const double*, S*, hipStream_t);       \
    template hipError_t launch_phase_init<S>(const PhaseK&, const double*, S*, hipStream_t);    \
    template hipError_t launch_chan_macros<S>(const ChanK&, const S*, double*, hipStream_t);    \
    template hipError_t launch_phase_macros<S>(const PhaseK&, const S*, double*, hipStream_t);  \
    template hipError_t launch_reduce<S>(int, const ChanK&, const PhaseK&, const D1K&,           \
                                         const D3K&, const P3K&, const S*, int, double*,          \
                                         double*, hipStream_t);                                   \
    template hipError_t launch_nonfinite_watch<S>(const S*, long long, long long, int, bool,     \
                                                  unsigned long long, unsigned long long*,       \
                                                  hipStream_t);                                   \
    template hipError_t launch_nusselt<S>(const ChanK&, const S*, const S*, double, double,      \
                                          double, double, int, double*, double*, double*, double*, \
                                          hipStream_t);
LBM_INST(float)
LBM_INST(double)

}  // namespace lbm

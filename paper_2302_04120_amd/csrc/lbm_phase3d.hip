// 3D two-phase step of liblbm for gfx950: the conservative Allen-Cahn h_i and
// the pressure-evolution z_i of Sec. 2.3 on D3Q19, z_i with the dimensional
// MRT of Sec. 3 in the d'Humieres basis, h_i BGK with its source.
//
// One step is two launches:
//   k_p3_phi   phi = sum_i h_i of the stored state into one plane (Eq.
//              zero_moment_h), so that no node has to re-read the 19 h_i of
//              its 18 neighbours;
//   k_p3_step  tiles of 64 x 4 x 1 nodes (FP32) or 64 x 2 x 2 (FP64); phi of
//              the tile and a one-node halo in LDS for the isotropic
//              stencils, then the node's collision in registers and push
//              streaming.
// Layout: node blocks (bidx, NPL3 values per node) with h 0-18, z 19-37, the
// low part of h_0 at 38 (FP32 storage: the rest population is an FP32 hi/lo
// pair that carries the node's exact phi balance, as in 2D), then (phi u) of
// the previous step (3 values); phi is one plain array of nodes.
// Arithmetic is lattice-normalised as in the 2D kernels: velocities / c,
// forces F dt^2 / dx, z_i in units of p / c_s^2, rates Lambda dt.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm_d3q19.h"
#include "lbm_device.h"

namespace lbm {
namespace {

// values per node of the 3D two-phase state: 42 in FP32 storage, 41 in FP64
template <typename S>
constexpr int NPL3 = std::is_same<S, float>::value ? 42 : 41;
template <typename S>
__device__ __forceinline__ long long p3idx(int i, long long n) {
    return bidx(NPL3<S>, i, n);
}

// Step tiles, measured on the 256^3 bubble box (ms per step, FP32 / FP64):
// 64 x 4 x 2 1.507 / 2.936, 64 x 2 x 2 1.498 / 2.806, 64 x 4 x 1 1.473 /
// 2.849, 64 x 2 x 4 1.514 / 2.912, 64 x 1 x 4 1.504 / 2.811, 64 x 8 x 1
// 1.568, 1024-thread tiles 1.58-1.62 / 3.59.  The states do not depend on
// the tiling.
template <typename S>
struct P3Tile {
    static constexpr int X = 64, Y = std::is_same<S, float>::value ? 4 : 2,
                         Z = std::is_same<S, float>::value ? 1 : 2;
    static constexpr int HX = X + 2, HY = Y + 2, HZ = Z + 2;
    static constexpr int Halo = HX * HY * HZ;  // phi values in LDS
    static constexpr int Threads = X * Y * Z;
};

__device__ __forceinline__ float rcp3(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp3(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq3(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq3(double x) { return 1.0 / sqrt(x); }

// phi of a node from its h_i (with the low part of h_0): one summation order
// everywhere
template <typename C>
__device__ __forceinline__ C phi_sum19(const C (&h)[19], C hlo) {
    const C ax = (h[1] + h[2]) + ((h[3] + h[4]) + (h[5] + h[6]));
    const C dg = ((h[7] + h[8]) + (h[9] + h[10])) + ((h[11] + h[12]) + (h[13] + h[14])) +
                 ((h[15] + h[16]) + (h[17] + h[18]));
    return (h[0] + hlo) + (ax + dg);
}

// index of a halo coordinate: periodic wrap, or at a wall the first fluid
// node (zero normal gradient of phi, as in 2D).  Halo coordinates of a ragged
// last tile can lie far beyond n (they feed no node but are still loaded),
// hence the full modulo.
__device__ __forceinline__ int ghost(int v, int n, int walls) {
    if (walls) return v < 0 ? 0 : (v >= n ? n - 1 : v);
    return ((v % n) + n) % n;
}

template <typename S>
__global__ __launch_bounds__(256) void k_p3_phi(P3K k, const S* __restrict__ a,
                                                S* __restrict__ phi) {
    constexpr bool RMASS = std::is_same<S, float>::value;
    const long long N = (long long)k.batch * k.nx * k.ny * k.nz;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        S h[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) h[i] = a[p3idx<S>(i, n)];
        phi[n] = phi_sum19<S>(h, RMASS ? a[p3idx<S>(38, n)] : S(0));
    }
}

// Everything one node does once phi of itself and its 18 neighbours is known
// (pn[i] = phi at x + e_i): stencils, macros, both collisions and the push
// of its populations into b -- or, with MACROS, its macroscopic fields into
// mout.  Shared by both step kernels, so that they agree to the last bit.
template <typename S, bool MACROS>
__device__ __forceinline__ void p3_node(const P3K& k, const S (&pn)[19], const S (&h)[19], S hlo,
                                        const S (&zz)[19], const S (&pu)[3], long long n, int x,
                                        int y, int z, long long base, S* __restrict__ b,
                                        double* __restrict__ mout, long long P) {
    using C = S;
    constexpr bool RMASS = std::is_same<S, float>::value;
    constexpr int PU = RMASS ? 39 : 38;  // first (phi u) plane
    const int nx = k.nx, ny = k.ny, nz = k.nz;
    const long long plane = (long long)nx * ny;
    // ---- stencils (Eq. gradient, Eq. laplacian): grad phi = 3 G / dx,
    //      lap phi = 6 L / dx^2
    const C phi = pn[0];
    C G[3] = {C(0), C(0), C(0)}, Lp = C(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const C wp = w19<C>(i) * pn[i];
        G[0] += C(E3X[i]) * wp;
        G[1] += C(E3Y[i]) * wp;
        G[2] += C(E3Z[i]) * wp;
        Lp += w19<C>(i) * (pn[i] - phi);
    }
    const C drl = C(k.rho_l - k.rho_g);
    const C rho = C(k.rho_g) + phi * drl;
    const C ir = rcp3(rho);
    C wn;
    if (k.visc_mode == 0) {
        wn = rcp3(C(3) * (C(k.nuh_g) + phi * C(k.nuh_l - k.nuh_g)) + C(0.5));
    } else {
        const C zh = C(k.zh_g) + phi * C(k.zh_l - k.zh_g);
        wn = rho * rcp3(C(3) * zh + C(0.5) * rho);
    }
    // chemical potential (Eq. chemical_potential), force mu grad phi + F_b
    const C mu = C(4) * C(k.beta) * phi * (phi - C(1)) * (phi - C(0.5)) - C(k.kap6) * Lp;
    C F[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) F[c] = mu * G[c] * C(k.fs_scale) + C(k.Fbt[c]);
    // guarded interface normal
    const C gn2 = (G[0] * G[0] + G[1] * G[1]) + G[2] * G[2];
    C nv[3] = {C(0), C(0), C(0)};
    if (gn2 > C(k.Geps) * C(k.Geps)) {
        const C ig = rsq3(gn2);
#pragma unroll
        for (int c = 0; c < 3; ++c) nv[c] = G[c] * ig;
    }
    // velocity first (Eq. u_Liang), then pressure (Eq. p_Liang) with w_0 = 1/3:
    // p / c_s^2 = 3/2 [sum_{i>0} z_i + 3/2 drho u.G - rho u^2 / 2]
    C m[19];
    moments19(zz, m);
    C u[3];
    u[0] = (m[3] + C(0.5) * F[0]) * ir;
    u[1] = (m[5] + C(0.5) * F[1]) * ir;
    u[2] = (m[7] + C(0.5) * F[2]) * ir;
    const C uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    const C ug = (u[0] * G[0] + u[1] * G[1]) + u[2] * G[2];
    const C zsum = ((zz[1] + zz[2]) + ((zz[3] + zz[4]) + (zz[5] + zz[6]))) +
                   (((zz[7] + zz[8]) + (zz[9] + zz[10])) + ((zz[11] + zz[12]) + (zz[13] + zz[14])) +
                    ((zz[15] + zz[16]) + (zz[17] + zz[18])));
    const C ph = C(1.5) * (zsum + C(1.5) * drl * ug - C(0.5) * rho * uu);

    if constexpr (MACROS) {
        mout[n] = double(rho);
        mout[P + n] = double(ph) * k.cs2;
        mout[2 * P + n] = double(u[0]) * k.c;
        mout[3 * P + n] = double(u[1]) * k.c;
        mout[4 * P + n] = 0.0;
        mout[5 * P + n] = double(phi);
        mout[6 * P + n] = double(mu);
        mout[7 * P + n] = double(u[2]) * k.c;
        return;
    } else {
        // ---- interface populations (Eq. eq_lattice_boltzmann_interface,
        //      source_term_interface, heq_liang); d(phi u)/dt by explicit Euler
        C dp[3], pn3[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pn3[c] = phi * u[c];
            dp[c] = pn3[c] - pu[c];
        }
        const C wphi = C(k.w_phi);
        const C sfac = C(1) - C(0.5) * wphi;
        const C sharp = C(4) * phi * (C(1) - phi) * C(k.dxW);
        const C A[3] = {C(3) * dp[0] + sharp * nv[0], C(3) * dp[1] + sharp * nv[1],
                        C(3) * dp[2] + sharp * nv[2]};
        C hs[19];
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            const C eu = (C(E3X[i]) * u[0] + C(E3Y[i]) * u[1]) + C(E3Z[i]) * u[2];
            const C eA = (C(E3X[i]) * A[0] + C(E3Y[i]) * A[1]) + C(E3Z[i]) * A[2];
            const C heq = phi * w19<C>(i) * (C(1) + C(3) * eu);
            hs[i] = h[i] - wphi * (h[i] - heq) + sfac * w19<C>(i) * eA;
        }
        S h0hi, h0lo = S(0);
        if constexpr (RMASS) {
            // rest population: the node's exact balance phi - sum_{i>0} h_i* with
            // the stored (rounded) h_i*, summed in FP64, kept as an FP32 pair
            double acc = double(h[0]) + double(hlo);
#pragma unroll
            for (int i = 1; i < 19; ++i) acc += double(h[i]);
#pragma unroll
            for (int i = 1; i < 19; ++i) acc -= double(float(hs[i]));
            h0hi = float(acc);
            h0lo = float(acc - double(h0hi));
        } else {
            h0hi = S(h[0] - wphi * (h[0] - phi * w19<C>(0)));
        }
        // ---- pressure collision in moment space.  Moments of z^eq (Eq.
        //      zeq_liang) and of dt F^z (Eq. forcing_term_pressure_evolution)
        //      in the D3Q19 basis, with p~ = p / c_s^2, D_ab = drho u_a G_b:
        //        m^eq = (0, 19 p~ + 19 rho u^2, -9 p~ - 11/2 rho u^2, rho u, -2/3 rho u,
        //                rho (2ux^2 - uy^2 - uz^2), -1/2 (.), rho (uy^2 - uz^2), -1/2 (.),
        //                rho ux uy, rho uy uz, rho ux uz, 0, 0, 0)
        //        m^F  = (3 D, 5 D, -2 D, F, -2/3 F, 2 (2Dxx - Dyy - Dzz), -(.),
        //                2 (Dyy - Dzz), -(.), Dxy + Dyx, Dyz + Dzy, Dxz + Dzx, 0, 0, 0)
        //      (j and q interleaved per axis as in the basis order).
        const C ruu = rho * uu;
        const C Dt = drl * ug;
        const C Dxx = drl * u[0] * G[0], Dyy = drl * u[1] * G[1], Dzz = drl * u[2] * G[2];
        const C pxx = rho * (C(2) * u[0] * u[0] - (u[1] * u[1] + u[2] * u[2]));
        const C pww = rho * (u[1] * u[1] - u[2] * u[2]);
        const C fxx = C(2) * Dxx - (Dyy + Dzz), fww = Dyy - Dzz;
        const C c23 = C(2) / C(3);
        const C meq[19] = {C(0), C(19) * (ph + ruu), C(-9) * ph - C(5.5) * ruu,
                           rho * u[0], -c23 * rho * u[0], rho * u[1], -c23 * rho * u[1],
                           rho * u[2], -c23 * rho * u[2], pxx, C(-0.5) * pxx, pww, C(-0.5) * pww,
                           rho * u[0] * u[1], rho * u[1] * u[2], rho * u[0] * u[2],
                           C(0), C(0), C(0)};
        const C mf[19] = {C(3) * Dt, C(5) * Dt, C(-2) * Dt, F[0], -c23 * F[0], F[1], -c23 * F[1],
                          F[2], -c23 * F[2], C(2) * fxx, -fxx, C(2) * fww, -fww,
                          drl * (u[0] * G[1] + u[1] * G[0]), drl * (u[1] * G[2] + u[2] * G[1]),
                          drl * (u[0] * G[2] + u[2] * G[0]), C(0), C(0), C(0)};
        // rates (times dt): 1 on rho, e, eps, j, pi; w_q2 on q and m; dt/tau on
        // the stresses (Sec. 3's two-phase choice row by row); BGK: all dt/tau
        const C wq = C(3) * (C(2) - wn) * rcp3(C(3) - wn);
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const bool stress = q == 9 || q == 11 || q == 13 || q == 14 || q == 15;
            const bool odd3 = q == 4 || q == 6 || q == 8 || q >= 16;
            const C Lq = !k.z_mrt ? wn : (stress ? wn : (odd3 ? wq : C(1)));
            m[q] += -Lq * (m[q] - meq[q]) + (C(1) - C(0.5) * Lq) * mf[q];
        }
        C zs[19];
        inverse19(m, zs);

        // ---- stores: (phi u), the rest populations, then push streaming with
        //      halfway bounce-back on walled axes
#pragma unroll
        for (int c = 0; c < 3; ++c) st(b + p3idx<S>(PU + c, n), S(pn3[c]));
        st(b + p3idx<S>(0, n), h0hi);
        if constexpr (RMASS) st(b + p3idx<S>(38, n), h0lo);
        st(b + p3idx<S>(19, n), S(zs[0]));
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            const int txd = x + E3X[i], tyd = y + E3Y[i], tzd = z + E3Z[i];
            const bool out = (k.bcx && (txd < 0 || txd >= nx)) || (k.bcy && (tyd < 0 || tyd >= ny)) ||
                             (k.bcz && (tzd < 0 || tzd >= nz));
            if (out) {
                st(b + p3idx<S>(OPP3[i], n), S(hs[i]));
                st(b + p3idx<S>(19 + OPP3[i], n), S(zs[i]));
            } else {
                const long long d = base + (long long)wrap(tzd, nz) * plane +
                                    (long long)wrap(tyd, ny) * nx + wrap(txd, nx);
                st(b + p3idx<S>(i, d), S(hs[i]));
                st(b + p3idx<S>(19 + i, d), S(zs[i]));
            }
        }
    }
}

// One step (or, with MACROS, the macroscopic fields of the stored state).
template <typename S, bool MACROS>
__global__ __launch_bounds__(P3Tile<S>::Threads) void k_p3_step(P3K k, const S* __restrict__ a,
                                                        S* __restrict__ b,
                                                        const S* __restrict__ phig,
                                                        double* __restrict__ mout) {
    using C = S;
    constexpr bool RMASS = std::is_same<S, float>::value;
    constexpr int PU = RMASS ? 39 : 38;  // first (phi u) plane
    using T = P3Tile<S>;
    constexpr int kPX = T::X, kPY = T::Y, kPZ = T::Z, kHX = T::HX, kHY = T::HY;
    __shared__ C sphi[T::HZ][T::HY][T::HX];
    const int nx = k.nx, ny = k.ny, nz = k.nz;
    const long long P = k.P;
    const int gx = (nx + kPX - 1) / kPX, gy = (ny + kPY - 1) / kPY, gz = (nz + kPZ - 1) / kPZ;
    int tile;
    if (!xcd_tile(gx * gy * gz * k.batch, tile)) return;  // whole workgroup, before the barrier
    const int per = gx * gy * gz;
    const int bb = tile / per, r = tile - bb * per;
    const int x0 = (r % gx) * kPX, y0 = ((r / gx) % gy) * kPY, z0 = (r / (gx * gy)) * kPZ;
    const long long plane = (long long)nx * ny;
    const long long base = (long long)bb * nz * plane;
    const int tx = threadIdx.x, ty = threadIdx.y, tz = threadIdx.z;
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    const bool valid = x < nx && y < ny && z < nz;
    const long long n = base + (long long)z * plane + (long long)y * nx + x;

    // the node's own populations first, then the phi halo, then one barrier
    C h[19], zz[19], hlo = C(0), pu[3] = {C(0), C(0), C(0)};
    if (valid) {
#pragma unroll
        for (int i = 0; i < 19; ++i) h[i] = C(a[p3idx<S>(i, n)]);
#pragma unroll
        for (int i = 0; i < 19; ++i) zz[i] = C(a[p3idx<S>(19 + i, n)]);
        if (RMASS) hlo = C(a[p3idx<S>(38, n)]);
        if constexpr (!MACROS) {
#pragma unroll
            for (int c = 0; c < 3; ++c) pu[c] = C(a[p3idx<S>(PU + c, n)]);
        }
    }
    const int t = (tz * kPY + ty) * kPX + tx;
    for (int j = t; j < T::Halo; j += T::Threads) {
        const int hx = j % kHX, hy = (j / kHX) % kHY, hz = j / (kHX * kHY);
        const int gxx = ghost(x0 + hx - 1, nx, k.bcx);
        const int gyy = ghost(y0 + hy - 1, ny, k.bcy);
        const int gzz = ghost(z0 + hz - 1, nz, k.bcz);
        sphi[hz][hy][hx] = C(phig[base + (long long)gzz * plane + (long long)gyy * nx + gxx]);
    }
    __syncthreads();
    if (!valid) return;
    C pn[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) pn[i] = sphi[tz + 1 + E3Z[i]][ty + 1 + E3Y[i]][tx + 1 + E3X[i]];
    p3_node<S, MACROS>(k, pn, h, hlo, zz, pu, n, x, y, z, base, b, mout, P);
}


// equilibria from FP64 fields (staging slots 1 p, 2 ux, 3 uy, 7 uz, 5 phi)
template <typename S>
__global__ void k_p3_init(P3K k, const double* __restrict__ fld, S* __restrict__ a) {
    constexpr bool RMASS = std::is_same<S, float>::value;
    constexpr int PU = RMASS ? 39 : 38;
    const long long N = (long long)k.batch * k.nx * k.ny * k.nz;
    const long long P = k.P;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        const double p = fld[P + n], phi = fld[5 * P + n];
        const double u[3] = {fld[2 * P + n] / k.c, fld[3 * P + n] / k.c, fld[7 * P + n] / k.c};
        const double rho = k.rho_g + phi * (k.rho_l - k.rho_g);
        const double ph = p / k.cs2, uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double hsum = 0.0;
        for (int i = 1; i < 19; ++i) {
            const double eu = E3X[i] * u[0] + E3Y[i] * u[1] + E3Z[i] * u[2];
            const S hv = S(phi * w19<double>(i) * (1 + 3 * eu));
            a[p3idx<S>(i, n)] = hv;
            hsum += double(hv);
        }
        const double h0 = phi - hsum;  // the rest population closes phi exactly
        const S hi = S(h0);
        a[p3idx<S>(0, n)] = hi;
        if (RMASS) a[p3idx<S>(38, n)] = S(h0 - double(hi));
        for (int i = 0; i < 19; ++i) {
            const double eu = E3X[i] * u[0] + E3Y[i] * u[1] + E3Z[i] * u[2];
            const double w = w19<double>(i);
            a[p3idx<S>(19 + i, n)] =
                S(ph * (i == 0 ? w - 1 : w) + rho * w * (3 * eu + 4.5 * eu * eu - 1.5 * uu));
        }
        for (int c = 0; c < 3; ++c) a[p3idx<S>(PU + c, n)] = S(phi * u[c]);
    }
}

inline unsigned grid_p3(long long N, int bs) {
    long long g = (N + bs - 1) / bs;
    if (g > 65535LL * 16) g = 65535LL * 16;
    return unsigned(g < 1 ? 1 : g);
}

template <typename S>
hipError_t launch_phi(const P3K& k, const S* a, S* phi, hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny * k.nz;
    hipLaunchKernelGGL(k_p3_phi<S>, dim3(grid_p3(N, 256)), dim3(256), 0, s, k, a, phi);
    return hipGetLastError();
}

template <typename S>
long long p3_tiles(const P3K& k) {
    using T = P3Tile<S>;
    return (long long)((k.nx + T::X - 1) / T::X) * ((k.ny + T::Y - 1) / T::Y) *
           ((k.nz + T::Z - 1) / T::Z) * k.batch;
}

}  // namespace

template <typename S>
hipError_t launch_p3_step(const P3K& k, const S* a, S* b, S* phi, hipStream_t s) {
    hipError_t e = launch_phi<S>(k, a, phi, s);
    if (e != hipSuccess) return e;
    const long long tiles = p3_tiles<S>(k);
    dim3 blk(P3Tile<S>::X, P3Tile<S>::Y, P3Tile<S>::Z), grd(unsigned((tiles + kXCD - 1) / kXCD * kXCD));
    hipLaunchKernelGGL((k_p3_step<S, false>), grd, blk, 0, s, k, a, b, (const S*)phi,
                       (double*)nullptr);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_p3_init(const P3K& k, const double* fields, S* a, hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny * k.nz;
    hipLaunchKernelGGL(k_p3_init<S>, dim3(grid_p3(N, 256)), dim3(256), 0, s, k, fields, a);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_p3_macros(const P3K& k, const S* a, S* phi, double* out, hipStream_t s) {
    hipError_t e = launch_phi<S>(k, a, phi, s);
    if (e != hipSuccess) return e;
    const long long tiles = p3_tiles<S>(k);
    dim3 blk(P3Tile<S>::X, P3Tile<S>::Y, P3Tile<S>::Z), grd(unsigned((tiles + kXCD - 1) / kXCD * kXCD));
    hipLaunchKernelGGL((k_p3_step<S, true>), grd, blk, 0, s, k, a, (S*)nullptr, (const S*)phi, out);
    return hipGetLastError();
}

#define LBM_P3_INST(S)                                                                       \
    template hipError_t launch_p3_step<S>(const P3K&, const S*, S*, S*, hipStream_t);        \
    template hipError_t launch_p3_init<S>(const P3K&, const double*, S*, hipStream_t);       \
    template hipError_t launch_p3_macros<S>(const P3K&, const S*, S*, double*, hipStream_t);
LBM_P3_INST(float)
LBM_P3_INST(double)

}  // namespace lbm

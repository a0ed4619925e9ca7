// D3Q19 momentum step of liblbm for gfx950: the dimensional MRT of Sec. 3 in
// three dimensions (the extension the paper's conclusions call direct), BGK
// as the case of equal rates, Guo forcing, and per axis periodic or halfway
// bounce-back walls (Eq. BB_vel with u_w = 0).
//
// Layout and streaming follow the two-phase D2Q9 kernels: node n = ((b * nz +
// z) * ny + y) * nx + x, the 19 populations in node blocks (value i of node n
// at bidx(19, i, n); a wave's 64 nodes are one contiguous block), the stored
// state is the pre-collision set, and each node pushes its post-collision
// values to x + e_i (or back into its own opposite slot through a wall).
// FP32 storage keeps f_i - w_i rho_ref.
//
// Moment space.  The basis is the orthogonal set of d'Humieres et al. (2002)
// (rows rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww,
// p_xy, p_yz, p_xz, m_x, m_y, m_z).  The dimensional matrix scales row k by
// c^order(k); a diagonal relaxation commutes with that scaling, so the kernel
// works in lattice-normalised form (u / c, F dt^2 / dx, Lambda dt) and gets
// the populations of the dimensional scheme.  The equilibrium and forcing
// moments are closed forms, so neither feq_i nor the Guo term is built per
// population.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm_d3q19.h"
#include "lbm_device.h"

// Rows of 64 nodes per workgroup.  Measured on the 256^3 box with the state in
// node blocks (ms per FP32 step): 64 x 4 0.489, 64 x 2 0.490, 64 x 1 0.497;
// FP64 0.937-0.942 for all three.  Capping residency at 4 waves per SIMD by
// an LDS reserve, which helped when the state was stored as planes (0.541 ->
// 0.522 ms), now costs time (64 x 4: 0.502-0.504 ms; 64 x 2 0.515, 64 x 1
// 0.505), so every workgroup takes only the LDS it uses (none).
#ifndef LBM_D3_TY
#define LBM_D3_TY 4
#endif

namespace lbm {
namespace {

constexpr int kD3Ty = LBM_D3_TY;  // rows of 64 nodes per workgroup

// One step: tiles of 64 x kD3Ty nodes in one z plane of one replica, numbered x
// fastest, then y, z and replica, and handed to the XCDs in contiguous bands
// (a tile's z neighbours, into which it pushes, sit gx * gy tiles away in the
// same band).
template <typename S>
__global__ __launch_bounds__(64 * kD3Ty) void k_d3_step(D3K k, const S* __restrict__ fc,
                                                 S* __restrict__ fn) {
    using C = S;
    const int nx = k.nx, ny = k.ny, nz = k.nz;
    const int gx = (nx + 63) / 64, gy = (ny + kD3Ty - 1) / kD3Ty;
    int tile;
    if (!xcd_tile(gx * gy * nz * k.batch, tile)) return;
    const int r = tile % (gx * gy);
    const int bz = tile / (gx * gy);  // b * nz + z
    const int z = bz % nz;
    const int x = (r % gx) * 64 + threadIdx.x;
    const int y = (r / gx) * kD3Ty + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const long long plane = (long long)nx * ny;
    const long long base = (long long)(bz - z) * plane;  // first node of the replica
    const long long n = base + (long long)z * plane + (long long)y * nx + x;

    C d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = C(fc[bidx(19, i, n)]);
    C m[19];
    moments19(d, m);
    // macros: rho = rho_ref + sum d (the deviations carry no momentum of their own)
    const C drho = m[0];
    const C rho = C(k.rho_ref) + drho;
    const C fx = C(k.Ft[0]), fy = C(k.Ft[1]), fz = C(k.Ft[2]);
    const C ir = C(1) / rho;
    const C ux = (m[3] + C(0.5) * fx) * ir;  // Eq. first_moment_f, over c
    const C uy = (m[5] + C(0.5) * fy) * ir;
    const C uz = (m[7] + C(0.5) * fz) * ir;

    // non-equilibrium moments m - m_eq; m_eq in deviation form (minus rho_ref M w)
    const C rxx = rho * ux * ux, ryy = rho * uy * uy, rzz = rho * uz * uz;
    const C ruu = (rxx + ryy) + rzz;
    const C pxx = C(2) * rxx - (ryy + rzz), pww = ryy - rzz;
    C neq[19];
    neq[0] = C(0);
    neq[1] = m[1] - (C(19) * ruu - C(11) * drho);
    neq[2] = m[2] - (C(3) * drho - C(5.5) * ruu);
    neq[3] = C(0);
    neq[4] = m[4] + (C(2) / C(3)) * (rho * ux);
    neq[5] = C(0);
    neq[6] = m[6] + (C(2) / C(3)) * (rho * uy);
    neq[7] = C(0);
    neq[8] = m[8] + (C(2) / C(3)) * (rho * uz);
    neq[9] = m[9] - pxx;
    neq[10] = m[10] + C(0.5) * pxx;
    neq[11] = m[11] - pww;
    neq[12] = m[12] + C(0.5) * pww;
    neq[13] = m[13] - rho * ux * uy;
    neq[14] = m[14] - rho * uy * uz;
    neq[15] = m[15] - rho * ux * uz;
    neq[16] = m[16];
    neq[17] = m[17];
    neq[18] = m[18];
    // moments of the Guo term (Eq. forcing_term): the u-derivative of m_eq along F
    const C uf = (ux * fx + uy * fy) + uz * fz;
    const C fxx = ux * fx, fyy = uy * fy, fzz = uz * fz;
    const C qxx = C(2) * fxx - (fyy + fzz), qww = fyy - fzz;
    C mf[19];
    mf[0] = C(0);
    mf[1] = C(38) * uf;
    mf[2] = C(-11) * uf;
    mf[3] = fx;
    mf[4] = (C(-2) / C(3)) * fx;
    mf[5] = fy;
    mf[6] = (C(-2) / C(3)) * fy;
    mf[7] = fz;
    mf[8] = (C(-2) / C(3)) * fz;
    mf[9] = C(2) * qxx;
    mf[10] = -qxx;
    mf[11] = C(2) * qww;
    mf[12] = -qww;
    mf[13] = ux * fy + uy * fx;
    mf[14] = uy * fz + uz * fy;
    mf[15] = ux * fz + uz * fx;
    mf[16] = C(0);
    mf[17] = C(0);
    mf[18] = C(0);
    // Eq. colisao_MRT: dm = -Lambda (m - m_eq) + (I - Lambda/2) dt F, rates times dt
    C dm[19], dv[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        const C L = C(k.L[q]);
        dm[q] = -L * neq[q] + (C(1) - C(0.5) * L) * mf[q];
    }
    inverse19(dm, dv);

    // streaming with halfway bounce-back where a wall closes the axis
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const C v = d[i] + dv[i];
        const int tx = x + E3X[i], ty = y + E3Y[i], tz = z + E3Z[i];
        const bool out = (k.bcx && (tx < 0 || tx >= nx)) || (k.bcy && (ty < 0 || ty >= ny)) ||
                         (k.bcz && (tz < 0 || tz >= nz));
        if (out) {
            st(fn + bidx(19, OPP3[i], n), S(v));
        } else {
            const long long t = base + (long long)wrap(tz, nz) * plane +
                                (long long)wrap(ty, ny) * nx + wrap(tx, nx);
            st(fn + bidx(19, i, t), S(v));
        }
    }
}

// equilibrium populations from FP64 fields (staging slots 0 rho, 2 ux, 3 uy,
// 7 uz; velocities in m/s)
template <typename S>
__global__ void k_d3_init(D3K k, const double* __restrict__ fld, S* __restrict__ f) {
    const long long N = (long long)k.batch * k.nx * k.ny * k.nz;
    const long long P = k.P;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        const double rho = fld[n];
        const double ux = fld[2 * P + n] / k.c, uy = fld[3 * P + n] / k.c, uz = fld[7 * P + n] / k.c;
        const double uu = ux * ux + uy * uy + uz * uz;
        for (int i = 0; i < 19; ++i) {
            const double eu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
            f[bidx(19, i, n)] = S(w19<double>(i) * ((rho - k.rho_ref) + rho * (3 * eu + 4.5 * eu * eu - 1.5 * uu)));
        }
    }
}

// FP64 macros of the stored state into staging slots 0 rho, 2 ux, 3 uy, 7 uz
template <typename S>
__global__ void k_d3_macros(D3K k, const S* __restrict__ f, double* __restrict__ out) {
    const long long N = (long long)k.batch * k.nx * k.ny * k.nz;
    const long long P = k.P;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        double d[19], m[19];
        for (int i = 0; i < 19; ++i) d[i] = double(f[bidx(19, i, n)]);
        moments19(d, m);
        const double rho = k.rho_ref + m[0];
        out[n] = rho;
        out[2 * P + n] = (m[3] + 0.5 * k.Ft[0]) / rho * k.c;
        out[3 * P + n] = (m[5] + 0.5 * k.Ft[1]) / rho * k.c;
        out[7 * P + n] = (m[7] + 0.5 * k.Ft[2]) / rho * k.c;
    }
}

inline unsigned grid_1d(long long N, int bs) {
    long long g = (N + bs - 1) / bs;
    if (g > 65535LL * 16) g = 65535LL * 16;
    return unsigned(g < 1 ? 1 : g);
}

}  // namespace

long long d3_tiles(const D3K& k) {
    return (long long)((k.nx + 63) / 64) * ((k.ny + kD3Ty - 1) / kD3Ty) * k.nz * k.batch;
}

template <typename S>
hipError_t launch_d3_step(const D3K& k, const S* fc, S* fn, hipStream_t s) {
    const long long tiles = d3_tiles(k);
    dim3 blk(64, kD3Ty), grd(unsigned((tiles + kXCD - 1) / kXCD * kXCD));
    hipLaunchKernelGGL(k_d3_step<S>, grd, blk, 0, s, k, fc, fn);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_d3_init(const D3K& k, const double* fields, S* f, hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny * k.nz;
    hipLaunchKernelGGL(k_d3_init<S>, dim3(grid_1d(N, 256)), dim3(256), 0, s, k, fields, f);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_d3_macros(const D3K& k, const S* f, double* out, hipStream_t s) {
    const long long N = (long long)k.batch * k.nx * k.ny * k.nz;
    hipLaunchKernelGGL(k_d3_macros<S>, dim3(grid_1d(N, 256)), dim3(256), 0, s, k, f, out);
    return hipGetLastError();
}

#define LBM_D3_INST(S)                                                                   \
    template hipError_t launch_d3_step<S>(const D3K&, const S*, S*, hipStream_t);        \
    template hipError_t launch_d3_init<S>(const D3K&, const double*, S*, hipStream_t);   \
    template hipError_t launch_d3_macros<S>(const D3K&, const S*, double*, hipStream_t);
LBM_D3_INST(float)
LBM_D3_INST(double)

}  // namespace lbm

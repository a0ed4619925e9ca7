// Device helpers shared by the forward and adjoint kernels of liblbm:
// velocity sets, the integer moment transforms and their exact inverses, the
// XCD-aware tile numbering, and the node macros of the momentum populations.
// Included only by the library's .hip sources.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {
namespace {

// D2Q9: rest, E, N, W, S, NE, NW, SW, SE (Eq. velocity_D2Q9, weights_D2Q9)
__device__ constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// mirror images in y (same c_x, opposite c_y), for the symmetry plane
__device__ constexpr int MIRY[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
template <typename C>
__device__ __forceinline__ C wgt(int i) {
    return i == 0 ? C(4) / C(9) : (i < 5 ? C(1) / C(9) : C(1) / C(36));
}
// D2Q5 for temperature: rest 1/3, axes 1/6, c_s^2 = c^2/3
__device__ constexpr int EX5[5] = {0, 1, 0, -1, 0};
__device__ constexpr int EY5[5] = {0, 0, 1, 0, -1};
__device__ constexpr int OPP5[5] = {0, 3, 4, 1, 2};
__device__ constexpr int MIRY5[5] = {0, 1, 4, 3, 2};
template <typename C>
__device__ __forceinline__ C wgt5(int i) {
    return i == 0 ? C(1) / C(3) : C(1) / C(6);
}

// m = M v with the integer D2Q9 matrix (rows rho, e, eps, J_x, q_x, J_y, q_y,
// p_xx, p_xy of Eq. M_matrix), as sums and differences.
template <typename C>
__device__ __forceinline__ void moments9(const C v[9], C m[9]) {
    const C s14 = v[1] + v[2] + v[3] + v[4];
    const C s58 = v[5] + v[6] + v[7] + v[8];
    const C x13 = v[1] - v[3], y24 = v[2] - v[4];
    const C x58 = (v[5] - v[7]) + (v[8] - v[6]);
    const C y58 = (v[5] - v[7]) + (v[6] - v[8]);
    m[0] = v[0] + s14 + s58;
    m[1] = C(-4) * v[0] - s14 + C(2) * s58;
    m[2] = C(4) * v[0] - C(2) * s14 + s58;
    m[3] = x13 + x58;
    m[4] = C(-2) * x13 + x58;
    m[5] = y24 + y58;
    m[6] = C(-2) * y24 + y58;
    m[7] = (v[1] + v[3]) - (v[2] + v[4]);
    m[8] = (v[5] + v[7]) - (v[6] + v[8]);
}

// v = M^-1 m = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m
// (rows of M are orthogonal); computed from the exact inverse, not the
// printed one of App. A.
template <typename C>
__device__ __forceinline__ void inverse9(const C m[9], C v[9]) {
    const C a0 = m[0] * (C(1) / C(9)), a1 = m[1] * (C(1) / C(36)), a2 = m[2] * (C(1) / C(36));
    const C a3 = m[3] * (C(1) / C(6)), a4 = m[4] * (C(1) / C(12));
    const C a5 = m[5] * (C(1) / C(6)), a6 = m[6] * (C(1) / C(12));
    const C a7 = m[7] * C(0.25), a8 = m[8] * C(0.25);
    const C axis = a0 - a1 - C(2) * a2;     // common part of populations 1..4
    const C diag = a0 + C(2) * a1 + a2;     // common part of populations 5..8
    const C jx = a3 - C(2) * a4, jy = a5 - C(2) * a6;
    const C dx = a3 + a4, dy = a5 + a6;
    v[0] = a0 - C(4) * a1 + C(4) * a2;
    v[1] = axis + jx + a7;
    v[2] = axis + jy - a7;
    v[3] = axis - jx + a7;
    v[4] = axis - jy - a7;
    v[5] = diag + dx + dy + a8;
    v[6] = diag - dx + dy - a8;
    v[7] = diag - dx - dy + a8;
    v[8] = diag + dx - dy - a8;
}

// D2Q5 basis T, j_x, j_y, e, p_xx
template <typename C>
__device__ __forceinline__ void moments5(const C v[5], C m[5]) {
    const C s = v[1] + v[2] + v[3] + v[4];
    m[0] = v[0] + s;
    m[1] = v[1] - v[3];
    m[2] = v[2] - v[4];
    m[3] = C(-4) * v[0] + s;
    m[4] = (v[1] + v[3]) - (v[2] + v[4]);
}
template <typename C>
__device__ __forceinline__ void inverse5(const C m[5], C v[5]) {
    const C a0 = m[0] * C(0.2), a1 = m[1] * C(0.5), a2 = m[2] * C(0.5);
    const C a3 = m[3] * C(0.05), a4 = m[4] * C(0.25);
    v[0] = a0 - C(4) * a3;
    v[1] = a0 + a1 + a3 + a4;
    v[2] = a0 + a2 + a3 - a4;
    v[3] = a0 - a1 + a3 + a4;
    v[4] = a0 - a2 + a3 - a4;
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each with
// its own L2.  Renumber them so that XCD k walks the k-th contiguous band of
// tiles in order: a tile's neighbours (whose halo rows it reads and whose
// cache lines its shifted stores share) then run on the same XCD shortly
// before or after it.  Returns false for the padding workgroups of the last
// band.
constexpr int kXCD = 8;
__device__ __forceinline__ bool xcd_tile(int ntiles, int& t) {
    const int w = blockIdx.x;
    const int band = (ntiles + kXCD - 1) / kXCD;
    t = (w % kXCD) * band + w / kXCD;
    return t < ntiles;
}

// Stores of the next state: that buffer is read back only in the next step,
// after the whole state (far larger than the caches) has streamed through.
#ifndef LBM_NT_STORE
#define LBM_NT_STORE 0
#endif
template <typename T>
__device__ __forceinline__ void st(T* p, T v) {
#if LBM_NT_STORE
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

__device__ __forceinline__ int wrap(int v, int n) {
    if (v < 0) return v + n;
    if (v >= n) return v - n;
    return v;
}

// ---------------------------------------------------------------------------
// D2Q9 flow + D2Q5 temperature: one node per thread
// ---------------------------------------------------------------------------

// lattice-normalised macros of one node from its deviation populations d
template <typename C>
__device__ __forceinline__ void chan_flow_macros_v(const C d[9], C rho_ref, C ftx, C fty, C& drho,
                                                   C& rho, C& ux, C& uy) {
    drho = ((d[0] + (d[1] + d[3])) + (d[2] + d[4])) + ((d[5] + d[7]) + (d[6] + d[8]));
    rho = rho_ref + drho;
    const C jx = (d[1] - d[3]) + ((d[5] - d[7]) + (d[8] - d[6]));
    const C jy = (d[2] - d[4]) + ((d[5] - d[7]) + (d[6] - d[8]));
    const C ir = C(1) / rho;
    ux = (jx + C(0.5) * ftx) * ir;  // Eq. first_moment_f, divided by c
    uy = (jy + C(0.5) * fty) * ir;
}

// the same from the f values 0-8 of a node-blocked state of npl values per
// node (d receives them)
template <typename C, typename S>
__device__ __forceinline__ void chan_flow_macros(const S* __restrict__ f, int npl, long long n,
                                                 C rho_ref, C ftx, C fty, C d[9], C& drho,
                                                 C& rho, C& ux, C& uy) {
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = C(f[bidx(npl, i, n)]);
    chan_flow_macros_v<C>(d, rho_ref, ftx, fty, drho, rho, ux, uy);
}

// Lattice body force at a node whose temperature is T = T_ref + th: the
// constant force plus, when on, the Boussinesq force -rho_ref beta th g of
// Eq. buoyancy_force (App. D).
template <typename C>
__device__ __forceinline__ void chan_force(const ChanK& k, C th, C& fx, C& fy) {
    fx = C(k.Ft[0]);
    fy = C(k.Ft[1]);
    if (k.buoy) {
        fx += C(k.Bt[0]) * th;
        fy += C(k.Bt[1]) * th;
    }
}

}  // namespace
}  // namespace lbm

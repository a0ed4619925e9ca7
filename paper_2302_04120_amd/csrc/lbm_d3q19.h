// D3Q19 helpers shared by the 3D kernels of liblbm: the velocity set and its
// weights, and the integer moment transform of the d'Humieres et al. (2002)
// basis with its exact inverse.  Included only by the library's .hip sources.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {
namespace {

// velocity set: rest; +-x, +-y, +-z; the xy, xz and yz diagonals in
// opposite pairs (2k-1, 2k)
__device__ constexpr int E3X[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int E3Y[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int E3Z[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__device__ constexpr int OPP3[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

template <typename C>
__device__ __forceinline__ C w19(int i) {
    return i == 0 ? C(1) / C(3) : (i < 7 ? C(1) / C(18) : C(1) / C(36));
}

// m = M f with the integer D3Q19 basis, as sums and differences
template <typename C>
__host__ __device__ __forceinline__ void moments19(const C f[19], C m[19]) {
    const C ax = f[1] + f[2], ay = f[3] + f[4], az = f[5] + f[6];
    const C dx = f[1] - f[2], dy = f[3] - f[4], dz = f[5] - f[6];
    const C s7 = f[7] + f[8], d7 = f[7] - f[8], s9 = f[9] + f[10], d9 = f[9] - f[10];
    const C s11 = f[11] + f[12], d11 = f[11] - f[12], s13 = f[13] + f[14], d13 = f[13] - f[14];
    const C s15 = f[15] + f[16], d15 = f[15] - f[16], s17 = f[17] + f[18], d17 = f[17] - f[18];
    const C sxy = s7 + s9, sxz = s11 + s13, syz = s15 + s17;
    const C sa = (ax + ay) + az, sd = (sxy + sxz) + syz;
    // first moments of the diagonal groups: xy along x / y, xz along x / z, yz along y / z
    const C xy_x = d7 + d9, xy_y = d7 - d9;
    const C xz_x = d11 + d13, xz_z = d11 - d13;
    const C yz_y = d15 + d17, yz_z = d15 - d17;
    m[0] = (f[0] + sa) + sd;
    m[1] = C(-30) * f[0] + C(-11) * sa + C(8) * sd;
    m[2] = C(12) * f[0] + C(-4) * sa + sd;
    const C jdx = xy_x + xz_x, jdy = xy_y + yz_y, jdz = xz_z + yz_z;
    m[3] = dx + jdx;
    m[4] = C(-4) * dx + jdx;
    m[5] = dy + jdy;
    m[6] = C(-4) * dy + jdy;
    m[7] = dz + jdz;
    m[8] = C(-4) * dz + jdz;
    const C pa = C(2) * ax - (ay + az), pd = (sxy + sxz) - C(2) * syz;
    m[9] = pa + pd;
    m[10] = C(-2) * pa + pd;
    const C wa = ay - az, wd = sxy - sxz;
    m[11] = wa + wd;
    m[12] = C(-2) * wa + wd;
    m[13] = s7 - s9;
    m[14] = s15 - s17;
    m[15] = s11 - s13;
    m[16] = xy_x - xz_x;
    m[17] = yz_y - xy_y;
    m[18] = xz_z - yz_z;
}

// f = M^-1 m = M^T diag(1 / |row|^2) m (the rows are orthogonal)
template <typename C>
__host__ __device__ __forceinline__ void inverse19(const C m[19], C f[19]) {
    const C a0 = m[0] * (C(1) / C(19)), a1 = m[1] * (C(1) / C(2394)), a2 = m[2] * (C(1) / C(252));
    const C a3 = m[3] * C(0.1), a4 = m[4] * C(0.025);
    const C a5 = m[5] * C(0.1), a6 = m[6] * C(0.025);
    const C a7 = m[7] * C(0.1), a8 = m[8] * C(0.025);
    const C a9 = m[9] * (C(1) / C(36)), a10 = m[10] * (C(1) / C(72));
    const C a11 = m[11] * (C(1) / C(12)), a12 = m[12] * (C(1) / C(24));
    const C a13 = m[13] * C(0.25), a14 = m[14] * C(0.25), a15 = m[15] * C(0.25);
    const C a16 = m[16] * C(0.125), a17 = m[17] * C(0.125), a18 = m[18] * C(0.125);
    const C axis = (a0 - C(11) * a1) - C(4) * a2;
    const C diag = (a0 + C(8) * a1) + a2;
    const C p9 = a9 - C(2) * a10;   // 3p_xx pair on the axes: +-x get 2 (.), +-y/z get -(.)
    const C w11 = a11 - C(2) * a12; // p_ww pair on the axes
    const C pd = a9 + a10, wd = a11 + a12;
    f[0] = (a0 - C(30) * a1) + C(12) * a2;
    const C cx = axis + C(2) * p9, cy = (axis - p9) + w11, cz = (axis - p9) - w11;
    const C jx = a3 - C(4) * a4, jy = a5 - C(4) * a6, jz = a7 - C(4) * a8;
    f[1] = cx + jx;
    f[2] = cx - jx;
    f[3] = cy + jy;
    f[4] = cy - jy;
    f[5] = cz + jz;
    f[6] = cz - jz;
    const C bx = a3 + a4, by = a5 + a6, bz = a7 + a8;
    // xy diagonals
    {
        const C c0 = (diag + pd) + wd;
        const C X = bx + a16, Y = by - a17;
        f[7] = (c0 + a13) + (X + Y);
        f[8] = (c0 + a13) - (X + Y);
        f[9] = (c0 - a13) + (X - Y);
        f[10] = (c0 - a13) - (X - Y);
    }
    // xz diagonals
    {
        const C c0 = (diag + pd) - wd;
        const C X = bx - a16, Z = bz + a18;
        f[11] = (c0 + a15) + (X + Z);
        f[12] = (c0 + a15) - (X + Z);
        f[13] = (c0 - a15) + (X - Z);
        f[14] = (c0 - a15) - (X - Z);
    }
    // yz diagonals
    {
        const C c0 = diag - C(2) * pd;
        const C Y = by + a17, Z = bz - a18;
        f[15] = (c0 + a14) + (Y + Z);
        f[16] = (c0 + a14) - (Y + Z);
        f[17] = (c0 - a14) + (Y - Z);
        f[18] = (c0 - a14) - (Y - Z);
    }
}

}  // namespace
}  // namespace lbm

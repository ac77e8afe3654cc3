// FP64 3x3 blocks of the blob mobility and of the kinematic matrix, for the
// per-body preconditioner kernels (internal, device code).
#pragma once

#include <hip/hip_runtime.h>

namespace rmb {

// ---------------------------------------------------------------------------
// 3x3 pair block in FP64 (assembly of per-body blocks)
// ---------------------------------------------------------------------------

// 1 / sqrt(x) for x > 0: the hardware estimate and one third-order
// correction step, y (1 + e/2 + 3e^2/8) with e = 1 - x y^2.
__device__ __forceinline__ double blk_rsqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

// M_ij without the 1/(6 pi eta a) prefactor; row = velocity of i, column =
// force on j.  Same formulas as the pair kernels (eq:RPYTensor plus the
// wall image correction), with one inverse square root per distance and no
// division on the far branch.
__device__ inline void pair_block_f64(const double ri[3], const double rj[3], double a, bool wall,
                               double B[9]) {
    const double rx = ri[0] - rj[0], ry = ri[1] - rj[1], rz = ri[2] - rj[2];
    const double d2 = rx * rx + ry * ry + rz * rz;
    double ciso, crr;  // crr multiplies r r^T (already divided by d^2)
    if (d2 > 4.0 * a * a) {
        const double inv_d = blk_rsqrt(d2);
        const double t = a * inv_d, t2 = t * t;
        ciso = t * (0.75 + 0.5 * t2);
        crr = t * (0.75 - 1.5 * t2) * (inv_d * inv_d);
    } else if (d2 > 0.0) {
        const double inv_d = blk_rsqrt(d2), inv_a = 1.0 / a;
        ciso = 1.0 - 0.28125 * (d2 * inv_d) * inv_a;  // 1 - 9 d / (32 a)
        crr = 0.09375 * inv_a * inv_d;                  // 3 / (32 a d)
    } else {
        ciso = 1.0, crr = 0.0;  // a blob with itself
    }
    const double r[3] = {rx, ry, rz};
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) B[3 * p + q] = (p == q ? ciso : 0.0) + crr * r[p] * r[q];
    if (wall) {
        const double Rz = ri[2] + rj[2];
        const double invL = blk_rsqrt(rx * rx + ry * ry + Rz * Rz);
        const double e[3] = {rx * invL, ry * invL, Rz * invL};
        const double xw = a * invL, hh = rj[2] * invL, ez = e[2];
        const double xw2 = xw * xw, xw4 = xw2 * xw2, ez2 = ez * ez;
        const double T = hh * hh - ez * hh;
        const double c1 = 0.25 * xw * (-3.0 + 6.0 * T + xw2 * (6.0 * ez2 - 2.0) + xw4 * (2.0 - 10.0 * ez2));
        const double c2 = 0.25 * xw * (-3.0 - 18.0 * T + xw2 * (6.0 - 30.0 * ez2) + xw4 * (70.0 * ez2 - 10.0));
        const double c3 = xw * (1.5 * hh * (1.0 - 6.0 * ez2 + 6.0 * ez * hh) +
                                ez * (xw2 * (15.0 * ez2 - 3.0) + xw4 * (10.0 - 35.0 * ez2)));
        const double c4 = xw * (1.5 * hh - 5.0 * ez * xw4);
        const double c5 = xw * (-3.0 * (hh * hh + ez2 * xw2) + xw4 * (15.0 * ez2 - 2.0));
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q)
                B[3 * p + q] += (p == q ? c1 : 0.0) + c2 * e[p] * e[q] + (q == 2 ? c3 * e[p] : 0.0) +
                                (p == 2 ? c4 * e[q] : 0.0) + (p == 2 && q == 2 ? c5 : 0.0);
    }
}

// K_p row block of blob i: velocity of blob i per unit body motion U_p,
// K[c][k] for c in 0..2 (velocity component), k in 0..5 (u then omega):
// u_c + (omega x d)_c with d = r_i - q_p.
__device__ __forceinline__ double K_entry(const double d[3], int c, int k) {
    if (k < 3) return c == k ? 1.0 : 0.0;
    // (omega x d)_c = eps_{c,l,m} omega_l d_m ; derivative w.r.t. omega_l (l = k-3)
    const int l = k - 3;
    if (c == l) return 0.0;
    const int m = 3 - c - l;
    const double sgn = ((l - c + 3) % 3 == 1) ? 1.0 : -1.0;  // eps_{c,l,m}
    return sgn * d[m];
}

}  // namespace rmb

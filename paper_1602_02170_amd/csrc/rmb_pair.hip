// Blob-blob mobility product v = M lambda on gfx950 (Sec. 2.2.1).
//
// Pair block (eq:RPYTensor): for r = r_i - r_j, d = |r|,
//   far  (d > 2a):  C1 = 3a/(4d) + a^3/(2d^3),  C2 = 3a/(4d) - 3a^3/(2d^3)
//   near (d <= 2a): C3 = 1 - 9d/(32a),          C4 = 3d/(32a)
//   M_ij lambda_j = (6 pi eta a)^-1 [C_iso lambda_j + (C_rr/d^2)(r . lambda_j) r]
// Above a no-slip wall (Sec. 2.1.1, Sec. 5) the Rotne-Prager-Blake
// correction of the image system is added: with R = r_i - (x_j, y_j, -z_j),
// L = |R|, e = R/L, xi = a/L, hh = z_j/L, ez = e_z,
//   W f = (6 pi eta a)^-1 [c1 f + (c2 (e.f) + c3 f_z) e + (c4 (e.f) + c5 f_z) z]
// with c1..c5 polynomials in xi, hh, ez (the double-Faxen image of Blake's
// Green's function; coefficients written out where they are evaluated).
//
// Execution model.  One lane owns one target blob (positions kept in FP64
// registers); a workgroup holds 256 targets (4 wave64s).  Every lane of a
// wave visits the same source at the same time.  In the FP64 kernel here the
// source records are wave-uniform loads that the compiler serves from the
// scalar cache into SGPRs (no LDS staging, no barriers); the FP32 kernel
// stages its sources in LDS instead (pair_lds_f32_kernel), because FP32
// arithmetic with an SGPR operand issues at half the rate of the register
// form on gfx950.  The source range of a system is split
// into chunks so that small systems still launch thousands of workgroups;
// each chunk writes its own FP64 partial sum and a second pass adds the
// chunks in a fixed order (deterministic, independent of other systems in
// the same launch).
#include <cmath>

#include "rmb_common.h"

namespace rmb {

void split_plan_rect(int64_t nt, int64_t ns, int32_t *n_split, int64_t *chunk, int32_t *n_tblock) {
    int64_t T = std::max<int64_t>((nt + kPairBlock - 1) / kPairBlock, 1);
    // enough workgroups to fill 256 CUs several times over, and no source
    // chunk longer than 4096 blobs
    int64_t want = std::max<int64_t>((ns + 4095) / 4096, (4096 + T - 1) / T);
    int64_t maxs = (ns + kAccBlock - 1) / kAccBlock;
    want = std::min(std::max<int64_t>(want, 1), std::max<int64_t>(maxs, 1));
    int64_t c = (ns + want - 1) / want;
    c = std::max<int64_t>((c + kAccBlock - 1) / kAccBlock * kAccBlock, kAccBlock);
    *chunk = c;
    *n_split = (int32_t)std::max<int64_t>((ns + c - 1) / c, 1);
    *n_tblock = (int32_t)T;
}

void split_plan(int64_t nb, int32_t *n_split, int64_t *chunk, int32_t *n_tblock) {
    split_plan_rect(nb, nb, n_split, chunk, n_tblock);
}

void pair_job_init(PairJob *J, const double *tpos, const void *src, double *partial, int64_t nb,
                   double a) {
    pair_job_init_rect(J, tpos, nb, src, nb, partial, a);
}

void pair_job_init_rect(PairJob *J, const double *tpos, int64_t nt, const void *src, int64_t ns, double *partial,
                        double a) {
    J->tpos = tpos;
    J->src = src;
    J->partial = partial;
    J->nb = nt;
    J->ns = ns;
    J->tile_begin = 0;
    split_plan_rect(nt, ns, &J->n_split, &J->chunk, &J->n_tblock);
    J->a = a;
    J->four_a2 = 4.0 * a * a;
    J->k_near_iso = 9.0 / (32.0 * a);
    J->k_near_rr = 3.0 / (32.0 * a);
}

// ---------------------------------------------------------------------------
// packing of source records
// ---------------------------------------------------------------------------

__global__ void pack_f32_kernel(const double *__restrict__ pos, const double *__restrict__ lam,
                                int64_t nb, SrcF32 *__restrict__ src) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    SrcF32 r;
    r.x = pos[3 * j + 0];
    r.y = pos[3 * j + 1];
    r.z = pos[3 * j + 2];
    r.fx = (float)lam[3 * j + 0];
    r.fy = (float)lam[3 * j + 1];
    r.fz = (float)lam[3 * j + 2];
    r.zf = (float)r.z;
    src[j] = r;
}

__global__ void pack_f64_kernel(const double *__restrict__ pos, const double *__restrict__ lam,
                                int64_t nb, SrcF64 *__restrict__ src) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    SrcF64 r;
    r.x = pos[3 * j + 0];
    r.y = pos[3 * j + 1];
    r.z = pos[3 * j + 2];
    r.fx = lam[3 * j + 0];
    r.fy = lam[3 * j + 1];
    r.fz = lam[3 * j + 2];
    src[j] = r;
}

hipError_t launch_pack_sources(int precision, const double *pos, const double *lam, int64_t nb,
                               void *src, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    dim3 g((unsigned)((nb + 255) / 256)), b(256);
    if (precision == RMB_PREC_FP32_PAIRS)
        hipLaunchKernelGGL(pack_f32_kernel, g, b, 0, s, pos, lam, nb, (SrcF32 *)src);
    else
        hipLaunchKernelGGL(pack_f64_kernel, g, b, 0, s, pos, lam, nb, (SrcF64 *)src);
    return hipGetLastError();
}

__global__ void pack_table_kernel(const PackJob *__restrict__ jobs, int32_t n_jobs) {
    const int64_t w = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= w) lo = mid; else hi = mid - 1;
    }
    const PackJob &J = jobs[lo];
    const int64_t j = (w - J.wg_begin) * 256 + threadIdx.x;
    if (j >= J.nb) return;
    const gmem<const double> pos = as_global(J.pos), lam = as_global(J.lam);
    const double x = pos[3 * j], y = pos[3 * j + 1], z = pos[3 * j + 2];
    const double fx = lam[3 * j], fy = lam[3 * j + 1], fz = lam[3 * j + 2];
    if (J.precision == RMB_PREC_FP32_PAIRS) {
        const gmem<SrcF32> r = as_global((SrcF32 *)J.src) + j;
        r->x = x, r->y = y, r->z = z;
        r->fx = (float)fx, r->fy = (float)fy, r->fz = (float)fz, r->zf = (float)z;
    } else {
        const gmem<SrcF64> r = as_global((SrcF64 *)J.src) + j;
        r->x = x, r->y = y, r->z = z, r->fx = fx, r->fy = fy, r->fz = fz;
    }
}

__global__ void pack_sub_kernel(const double *__restrict__ pos, const double *__restrict__ lam, int64_t nb,
                                const double *__restrict__ off, int32_t n_sub, double a, int wall, int precision,
                                void *src, int *flag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nb * n_sub) return;
    const int64_t i = s / n_sub;
    const int k = (int)(s % n_sub);
    const gmem<const double> P = as_global(pos), F = as_global(lam), O = as_global(off);
    const double x = P[3 * i] + a * O[3 * k], y = P[3 * i + 1] + a * O[3 * k + 1],
                 z = P[3 * i + 2] + a * O[3 * k + 2];
    const double w = 1.0 / n_sub;
    const double fx = F[3 * i] * w, fy = F[3 * i + 1] * w, fz = F[3 * i + 2] * w;
    int bad = 0;
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) bad |= 1;
    if (wall && !(z > 0.0)) bad |= 2;
    if (bad) atomicOr(flag, bad);
    if (precision == RMB_PREC_FP32_PAIRS) {
        const gmem<SrcF32> r = as_global((SrcF32 *)src) + s;
        r->x = x, r->y = y, r->z = z;
        r->fx = (float)fx, r->fy = (float)fy, r->fz = (float)fz, r->zf = (float)z;
    } else {
        const gmem<SrcF64> r = as_global((SrcF64 *)src) + s;
        r->x = x, r->y = y, r->z = z, r->fx = fx, r->fy = fy, r->fz = fz;
    }
}

hipError_t launch_pack_sub_sources(int precision, const double *pos, const double *lam, int64_t nb, const double *off,
                                   int32_t n_sub, double a, int wall, void *src, int *flag, hipStream_t s) {
    const int64_t n = nb * n_sub;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_sub_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pos, lam, nb, off, n_sub,
                       a, wall, precision, src, flag);
    return hipGetLastError();
}

hipError_t launch_pack_table(const PackJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_table_kernel, dim3((unsigned)n_wg), dim3(256), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pair kernels
// ---------------------------------------------------------------------------

// Which system and which tile of it this workgroup serves (wave-uniform).
__device__ __forceinline__ int find_job(const PairJob *__restrict__ jobs, int32_t n_jobs,
                                        int64_t w) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_begin <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Source records live in global memory and are never written by the pair
// kernels; naming the address space lets the compiler serve wave-uniform
// reads of them through scalar loads.
template <typename T>
using global_ptr = const __attribute__((address_space(1))) T *;

// 1/sqrt(x) in FP64: hardware estimate (about 23 correct bits) followed by a
// third-order correction y (1 + e/2 + 3e^2/8), e = 1 - x y^2.
__device__ __forceinline__ double rsqrt_f64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

template <bool WALL>
__global__ __launch_bounds__(kPairBlock) void pair_f64_kernel(const PairJob *__restrict__ jobs,
                                                             int32_t n_jobs) {
    const int64_t w = blockIdx.x;
    const int k = find_job(jobs, n_jobs, w);
    const PairJob &J = jobs[k];
    const int64_t lt = w - J.tile_begin;
    const int32_t split = (int32_t)(lt / J.n_tblock);
    const int64_t t0 = (lt % J.n_tblock) * kPairBlock;
    const int64_t s0 = split * J.chunk;
    const int64_t s1 = min(s0 + J.chunk, J.ns);
    global_ptr<SrcF64> __restrict__ src = (global_ptr<SrcF64>)J.src;

    const int64_t i = t0 + threadIdx.x;
    const bool active = i < J.nb;
    const int64_t ii = active ? i : t0;
    const double xi = as_global(J.tpos)[3 * ii + 0], yi = as_global(J.tpos)[3 * ii + 1], zi = as_global(J.tpos)[3 * ii + 2];

    const double a = J.a, four_a2 = J.four_a2, kiso = J.k_near_iso, krr = J.k_near_rr;
    double ax = 0.0, ay = 0.0, az = 0.0;

#pragma unroll 2
    for (int64_t j = s0; j < s1; ++j) {
        SrcF64 s;
        s.x = src[j].x, s.y = src[j].y, s.z = src[j].z;
        s.fx = src[j].fx, s.fy = src[j].fy, s.fz = src[j].fz;
        const double rx = xi - s.x, ry = yi - s.y, rz = zi - s.z;
        const double rxy2 = fma(rx, rx, ry * ry);
        const double d2 = fma(rz, rz, rxy2);
        const double inv_d = rsqrt_f64(d2 + 1e-280);
        const double d = d2 * inv_d;
        const double t = a * inv_d;
        const double t2 = t * t;
        const double iso_far = t * fma(0.5, t2, 0.75);
        const double rr_far = t * fma(-1.5, t2, 0.75) * (inv_d * inv_d);
        const double iso_near = fma(-kiso, d, 1.0);
        const double rr_near = krr * inv_d;
        const bool near = d2 <= four_a2;
        const double ciso = near ? iso_near : iso_far;
        const double crr = near ? rr_near : rr_far;
        const double pxy = fma(rx, s.fx, ry * s.fy);
        const double sr = crr * fma(rz, s.fz, pxy);
        ax = fma(ciso, s.fx, fma(sr, rx, ax));
        ay = fma(ciso, s.fy, fma(sr, ry, ay));
        az = fma(ciso, s.fz, fma(sr, rz, az));
        if (WALL) {
            const double Rz = zi + s.z;
            const double L2 = fma(Rz, Rz, rxy2);
            const double invL = rsqrt_f64(L2);
            const double xw = a * invL, hh = s.z * invL, ez = Rz * invL;
            const double xw2 = xw * xw, xw4 = xw2 * xw2, ez2 = ez * ez;
            const double hh2 = hh * hh, ezh = ez * hh;
            const double T = hh2 - ezh;
            const double xq = 0.25 * xw;
            const double c1 = xq * fma(xw4, fma(-10., ez2, 2.),
                                       fma(xw2, fma(6., ez2, -2.), fma(6., T, -3.)));
            const double c2 = xq * fma(xw4, fma(70., ez2, -10.),
                                       fma(xw2, fma(-30., ez2, 6.), fma(-18., T, -3.)));
            const double hh15 = 1.5 * hh;
            const double m3 = hh15 * fma(-6., ez2, fma(6., ezh, 1.));
            const double e3 = fma(xw2, fma(15., ez2, -3.), xw4 * fma(-35., ez2, 10.));
            const double c3 = xw * fma(ez, e3, m3);
            const double c4 = xw * fma(-5. * ez, xw4, hh15);
            const double c5 = xw * fma(xw4, fma(15., ez2, -2.), -3. * fma(ez2, xw2, hh2));
            const double ef = fma(Rz, s.fz, pxy) * invL;
            const double g = fma(c2, ef, c3 * s.fz) * invL;
            const double kz = fma(c4, ef, c5 * s.fz);
            ax = fma(c1, s.fx, fma(g, rx, ax));
            ay = fma(c1, s.fy, fma(g, ry, ay));
            az = fma(c1, s.fz, fma(g, Rz, az)) + kz;
        }
    }
    if (active) {
        const gmem<double> out = as_global(J.partial + ((int64_t)split * J.nb + i) * 3);
        out[0] = ax;
        out[1] = ay;
        out[2] = az;
    }
}

hipError_t launch_pair_tiles(int precision, bool wall, const PairJob *jobs, int32_t n_jobs,
                             int64_t n_tiles, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    dim3 g((unsigned)n_tiles), b(kPairBlock);
    if (precision == RMB_PREC_FP32_PAIRS) {
        return launch_pair_lds_f32(wall, jobs, n_jobs, n_tiles, s);
    } else {
        if (wall)
            hipLaunchKernelGGL(pair_f64_kernel<true>, g, b, 0, s, jobs, n_jobs);
        else
            hipLaunchKernelGGL(pair_f64_kernel<false>, g, b, 0, s, jobs, n_jobs);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reduction of split partials, validation
// ---------------------------------------------------------------------------

__global__ void reduce_partials_kernel(const double *__restrict__ partial, int32_t n_split,
                                       int64_t n3, double pref, double *__restrict__ v) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    double acc = 0.0;
    for (int32_t s = 0; s < n_split; ++s) acc += partial[(int64_t)s * n3 + e];
    v[e] = pref * acc;
}

hipError_t launch_reduce_partials(const double *partial, int32_t n_split, int64_t nb, double pref,
                                  double *v, hipStream_t s) {
    int64_t n3 = 3 * nb;
    if (n3 <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s,
                       partial, n_split, n3, pref, v);
    return hipGetLastError();
}

__global__ void validate_positions_kernel(const double *__restrict__ pos, int64_t nb, int wall,
                                          const double *__restrict__ shift, int *__restrict__ flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    int f = 0;
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) f |= 1;
    if (wall && !(z > 0.0)) f |= 2;
    if (shift) {
        const double d = shift[i];
        if (!(d >= 0.0) || !isfinite(d)) f |= 32;
    }
    if (f) atomicOr(flag, f);
}

hipError_t launch_validate_positions(const double *pos, int64_t nb, int wall, const double *shift, int *flag,
                                     hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(validate_positions_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0,
                       s, pos, nb, wall, shift, flag);
    return hipGetLastError();
}

// v_i += d_i lambda_i: the permeable-body slip -d_i lambda_i moved to the
// operator side (eq:permeable_slip), i.e. d on the diagonal of M.
__global__ void add_shift_kernel(const double *__restrict__ shift, const double *__restrict__ lam, int64_t nb,
                                 double *__restrict__ v) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * nb) return;
    v[e] += shift[e / 3] * lam[e];
}

hipError_t launch_add_shift(const double *shift, const double *lam, int64_t nb, double *v, hipStream_t s) {
    if (nb <= 0 || !shift) return hipSuccess;
    hipLaunchKernelGGL(add_shift_kernel, dim3((unsigned)((3 * nb + 255) / 256)), dim3(256), 0, s, shift, lam, nb,
                       v);
    return hipGetLastError();
}

}  // namespace rmb

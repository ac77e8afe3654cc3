// Blob mobility product evaluating each pair block once (Sec. 2.2.1).
//
// The blob mobility is symmetric, M_ji = M_ij^T: the free-space RPY block is
// a symmetric function of r_i - r_j, and the wall-corrected tensor is
// reciprocal (the Faxen-corrected Blake Green's function, Sec. 2.1.1).  So
// one evaluation of the pair's coefficients serves both
//   v_i += M_ij lambda_j   and   v_j += M_ij^T lambda_i.
//
// Blobs are split into blocks of B (64..512, chosen from Nb alone).  One
// workgroup is one wave and owns one block pair (I <= J).  It walks the
// targets of block I in groups of 64 (one per lane) against the sources of
// block J in groups of 64:
//   * every lane holds one target and one source of the group; in 64 steps
//     the sources, together with their running sums of M_ij^T lambda_i, are
//     passed one lane along the wave (DPP wave rotation), so each lane meets
//     every source once and each source meets every target once;
//   * target side: each lane sums M_ij lambda_j in FP32 over the 64 sources
//     of a group and flushes to FP64;
//   * source side: after a full turn each source is back in its own lane,
//     and its FP32 sum over the 64 targets is added to an FP64 accumulator.
// Diagonal tiles (I == J) use the one-sided form over all ordered pairs,
// with the sources as wave-uniform records from the scalar cache.
// Every tile writes its target-side sums for block I and its source-side
// sums for block J to its own slots; a second kernel adds, for each blob, its
// tiles' contributions in a fixed order (bitwise reproducible, independent of
// what shares the launch).
#include <cmath>
#include <type_traits>

#include "rmb_body.h"

namespace rmb {

template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

// Tile t of a T x T upper triangle (row-major over I, then J >= I).
__device__ __forceinline__ void tile_ij(int64_t t, int32_t T, int32_t *I, int32_t *J) {
    // I = largest i with start(i) = i*T - i*(i-1)/2 <= t
    const double b = 2.0 * T + 1.0;
    int32_t i = (int32_t)floor((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
    if (i < 0) i = 0;
    if (i > T - 1) i = T - 1;
    auto start = [&](int64_t r) { return r * T - r * (r - 1) / 2; };
    while (i > 0 && start(i) > t) --i;
    while (i + 1 < T && start(i + 1) <= t) ++i;
    *I = i;
    *J = i + (int32_t)(t - start(i));
}

// One DPP step: x + x(shifted by `CTRL`), rows outside ROW_MASK and lanes
// shifted in from outside the row read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
    const int s = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true);
    return x + __int_as_float(s);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return x + __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Sum over the 64 lanes of a wave; the total lands in lane 63:
// row_shr 1, 2, 4, 8 leave each row's sum in its lane 15, then row_bcast:15
// and row_bcast:31 carry the row sums up to lane 63.
template <typename R>
__device__ __forceinline__ R wave_sum_to_63(R v) {
    v = dpp_add<0x111, 0xf>(v);
    v = dpp_add<0x112, 0xf>(v);
    v = dpp_add<0x114, 0xf>(v);
    v = dpp_add<0x118, 0xf>(v);
    v = dpp_add<0x142, 0xa>(v);
    v = dpp_add<0x143, 0xc>(v);
    return v;
}

// Moves a value one lane up the wave (lane l receives lane l-1, lane 0
// receives lane 63).  Every lane is written, so no prior value is needed.
__device__ __forceinline__ float rot1(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x13c, 0xf, 0xf, false));
}
__device__ __forceinline__ double rot1(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x13c, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x13c, 0xf, 0xf, false);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

template <typename R>
__device__ __forceinline__ R read_lane63(R v);
template <>
__device__ __forceinline__ float read_lane63(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
template <>
__device__ __forceinline__ double read_lane63(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

__device__ __forceinline__ double rsqrt64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}
// The result of a transcendental instruction needs one wait state before a
// VALU instruction reads it.  The compiler inserts it for its own consumers
// but not for the inline-asm consumers below, so the wait is part of the
// instruction's own asm.
__device__ __forceinline__ float rsqrt_r(float x) {
    float y;
    asm("v_rsq_f32_e32 %0, %1\n\ts_nop 0" : "=v"(y) : "v"(x));
    return y;
}
__device__ __forceinline__ double rsqrt_r(double x) { return rsqrt64(x); }

// x + y, not moved out of the branch it is written in.
__device__ __forceinline__ float add_in_place(float x, float y) {
    float d;
    asm volatile("v_add_f32_e64 %0, %1, %2" : "=v"(d) : "v"(x), "v"(y));
    return d;
}
__device__ __forceinline__ double add_in_place(double x, double y) { return x + y; }

// Arithmetic between two or three register operands.  On gfx950 the
// two-VGPR-source VOP2 encodings of v_mul/v_add/v_sub/v_fmac_f32 issue at
// about 21 lanes per clock per SIMD, while the same operations in VOP3
// encoding issue at 27-30, so the FP32 forms are written as VOP3 explicitly
// (the compiler would shrink them to VOP2).  Operations with a constant
// operand stay plain C: the compiler gives them literal or inline-constant
// forms, which also issue at about 30.  FP64 arithmetic is VOP3 only.
template <typename R>
struct VOp;
template <>
struct VOp<float> {
    static __device__ __forceinline__ float mul(float a, float b) {
        float d;
        asm("v_mul_f32_e64 %0, %1, %2" : "=v"(d) : "v"(a), "v"(b));
        return d;
    }
    static __device__ __forceinline__ float add(float a, float b) {
        float d;
        asm("v_add_f32_e64 %0, %1, %2" : "=v"(d) : "v"(a), "v"(b));
        return d;
    }
    static __device__ __forceinline__ float sub(float a, float b) {
        float d;
        asm("v_sub_f32_e64 %0, %1, %2" : "=v"(d) : "v"(a), "v"(b));
        return d;
    }
    static __device__ __forceinline__ float fma(float a, float b, float c) {
        float d;
        asm("v_fma_f32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
        return d;
    }
};
template <>
struct VOp<double> {
    static __device__ __forceinline__ double mul(double a, double b) { return a * b; }
    static __device__ __forceinline__ double add(double a, double b) { return a + b; }
    static __device__ __forceinline__ double sub(double a, double b) { return a - b; }
    static __device__ __forceinline__ double fma(double a, double b, double c) { return ::fma(a, b, c); }
};

// Coefficients of one pair block, shared by both contractions:
//   M_ij f   = A f + Bv (r . f) r + W f,   W f = c1 f + (c2 (e.f) + c3 f_z) e + (c4 (e.f) + c5 f_z) z
//   M_ij^T f = A f + Bv (r . f) r + c1 f + (c2 (e.f) + c4 f_z) e + (c3 (e.f) + c5 f_z) z
// with e = R / L.  The contractions take R . f unnormalised, so the stored
// image coefficients are c2 / L^2, c3 / L and c4 / L; and since R = r + 2 z_j z,
// the e-term shares the direction r with the RPY term in x and y, the z row
// taking the rest as g 2 z_j.
//
// Lengths are in units of the blob radius: the caller passes r / a and z_j / a
// (positions are scaled by 1/a in FP64 before they are rounded to the pair
// precision).  The RPY and image coefficients depend only on the ratios
// a / r, a / L and z_j / L, so the near-field constants become the pure
// numbers 9/32 and 3/32, the contact test is r^2 <= 4, a / L is the inverse
// square root itself, and the coefficients of the (r . f) r and R-terms come
// out as Bv a^2, c2 a^2 / L^2 and c_k a / L, which is what the scaled vectors
// need: the contractions return M_ij f unchanged.
template <typename R, bool WALL>
struct PairCoef {
    using P = VOp<R>;
    R iso, crr;              // ciso + c1 (ciso alone in free space), and crr: ciso I + crr r r^T
    R c2L, c3L, c4L, isoz;   // wall image: c2 / L^2, c3 / L, c4 / L; isoz = iso + c5 (the z-z diagonal)
    R Rz, zj2;               // R_z = r_z + 2 z_j, and 2 z_j

    // NEAR_POSSIBLE = false: the caller knows r > 2a (far branch only).
    template <bool NEAR_POSSIBLE = true>
    __device__ __forceinline__ void eval(R rx, R ry, R rz, R zj, R tiny) {
        const R rxy2 = P::fma(ry, ry, P::mul(rx, rx));
        const R d2 = P::fma(rz, rz, rxy2);
        eval_d2<NEAR_POSSIBLE>(rxy2, d2, rz, zj, zj + zj, tiny);
    }
    // zj2 = 2 z_j, passed in (the symmetric product stages it with the source)
    template <bool NEAR_POSSIBLE>
    __device__ __forceinline__ void eval_d2(R rxy2, R d2, R rz, R zj, R zj2_, R tiny) {
        // r = 0 (a blob with itself) only on the near branch; the far one has
        // r^2 > 4.  The guard is added in a form the compiler keeps inside
        // the near branch (hoisted, it would cost the far steps too).
        const R t = rsqrt_r(NEAR_POSSIBLE ? add_in_place(d2, tiny) : d2);  // a / r
        const R t2 = P::mul(t, t);
        const R iso_far = P::mul(t, (R)0.5 * t2 + (R)0.75);
        const R rr_far = P::mul(P::mul(t, t2), (R)-1.5 * t2 + (R)0.75);
        R ciso = iso_far;
        crr = rr_far;
        if (NEAR_POSSIBLE) {
            const R d = P::mul(d2, t);  // r / a
            const R iso_near = (R)1 - (R)(9.0 / 32.0) * d;
            const R rr_near = (R)(3.0 / 32.0) * t;
            const bool near = d2 <= (R)4;
            ciso = near ? iso_near : iso_far;
            crr = near ? rr_near : rr_far;
        }
        if (WALL) {
            zj2 = zj2_;
            Rz = zj2 + rz;
            const R L2 = P::fma(Rz, Rz, rxy2);
            const R xw = rsqrt_r(L2);  // a / L
            const R hh = P::mul(zj, xw), ez = P::mul(Rz, xw);
            const R xw2 = P::mul(xw, xw), xw4 = P::mul(xw2, xw2), ez2 = P::mul(ez, ez);
            const R hh2 = P::mul(hh, hh), ezh = P::mul(ez, hh);
            const R T = P::sub(hh2, ezh);
            const R xw3 = P::mul(xw, xw2);
            // c1 and c2 carry xi / 4, folded into their polynomials:
            //   c1 = xw q1, q1 = xw^4 (0.5 - 2.5 ez^2) + xw^2 (1.5 ez^2 - 0.5) + 1.5 T - 0.75
            //   c2 = xw q2, q2 = xw^4 (17.5 ez^2 - 2.5) + xw^2 (1.5 - 7.5 ez^2) - 4.5 T - 0.75
            // and q1 = -q2 / 5 + xw^4 ez^2 - 0.2 xw^2 + 0.6 T - 0.9
            const R q2 = P::fma(xw4, (R)17.5 * ez2 - (R)2.5, P::fma(xw2, (R)-7.5 * ez2 + (R)1.5, (R)-4.5 * T - (R)0.75));
            const R q1 = (R)-0.2 * q2 + P::fma(xw4, ez2, (R)-0.2 * xw2 + ((R)0.6 * T - (R)0.9));
            iso = P::fma(xw, q1, ciso);
            c2L = P::mul(xw3, q2);
            // c3 = xw^2 (ez e3 + m3) with e3 = xw^4 (10 - 35 ez^2) + xw^2 (15 ez^2 - 3)
            // and m3 = 1.5 hh (1 - 6 ez^2 + 6 ez hh) = 1.5 hh + 9 ez T; since
            // e3 + 9 T = 5 xw^4 - 2 q2 - 1.5, ez e3 + m3 = ez (5 xw^4 - 2 q2 - 1.5) + 1.5 hh
            const R hh15 = (R)1.5 * hh;
            c3L = P::mul(xw2, P::fma(ez, (R)-2 * q2 + ((R)5 * xw4 - (R)1.5), hh15));
            c4L = P::mul(xw2, P::fma((R)-5 * ez, xw4, hh15));
            isoz = P::fma(xw, P::fma(xw4, (R)15 * ez2 - (R)2, (R)-3 * P::fma(ez2, xw2, hh2)), iso);
        } else {
            iso = ciso;
        }
    }
    // out += M_ij f  (transpose = false) or M_ij^T f (transpose = true)
    template <bool TRANSPOSE>
    __device__ __forceinline__ void apply(R rx, R ry, R rz, R fx, R fy, R fz, R &ox, R &oy, R &oz) const {
        const R pxy = P::fma(ry, fy, P::mul(rx, fx));
        const R rf = P::fma(rz, fz, pxy);
        if (!WALL) {
            const R sr = P::mul(crr, rf);
            ox = P::fma(iso, fx, P::fma(sr, rx, ox));
            oy = P::fma(iso, fy, P::fma(sr, ry, oy));
            oz = P::fma(iso, fz, P::fma(sr, rz, oz));
        } else {
            const R Rf = P::fma(Rz, fz, pxy);
            const R ce = TRANSPOSE ? c4L : c3L, cz = TRANSPOSE ? c3L : c4L;
            const R g = P::fma(c2L, Rf, P::mul(ce, fz));
            const R gr = P::fma(crr, rf, g);
            ox = P::fma(iso, fx, P::fma(gr, rx, ox));
            oy = P::fma(iso, fy, P::fma(gr, ry, oy));
            oz = P::fma(isoz, fz, P::fma(gr, rz, P::fma(g, zj2, P::fma(cz, Rf, oz))));
        }
    }
};

template <typename SRC>
struct SrcView;
template <>
struct SrcView<SrcF32> {
    using R = float;
};
template <>
struct SrcView<SrcF64> {
    using R = double;
};


// A group of 64 sources staged in LDS twice over (entries l and l + 64 hold
// source l), so that lane l reads the source it pairs with at step s at
// entry l - s + 64 without wrapping.
template <typename R>
struct SymStage;
// FP32 pairs: positions as two floats, p = hi + lo with hi = fl32(p) and
// lo = fl32(p - hi).  The difference of two positions is then formed as
// (hi_i - hi_j) + (lo_i - lo_j) in FP32: the hi difference is exact when the
// two coordinates are within a factor of two of each other (Sterbenz) and
// otherwise rounded once at the scale of the result, the lo difference
// carries an error of about 2^-48 |p|, so the result matches the FP64
// difference rounded to FP32 to within an ulp, without FP64 arithmetic.
struct Pos2 {
    float xh, yh, zh, xl, yl, zl;
    __device__ __forceinline__ void set(double x, double y, double z) {
        xh = (float)x, yh = (float)y, zh = (float)z;
        xl = (float)(x - (double)xh), yl = (float)(y - (double)yh), zl = (float)(z - (double)zh);
    }
};

struct Pos64 {
    double v[3];
    double ia;  // 1/a: FP64 differences are formed from physical positions, then scaled
};

template <>
struct SymStage<float> {
    float2 xy[128], zx[128], yz[128], fxy[128], fz[128];  // (xh, yh), (zh, xl), (yl, zl), (fx, fy), (fz, 2 zh)
    // positions already in units of a (zs, the same height, unused here)
    __device__ __forceinline__ void put(int l, double px, double py, double pz, float fx, float fy, float gz,
                                        double /*zs*/) {
        Pos2 q;
        q.set(px, py, pz);
        xy[l] = xy[l + 64] = make_float2(q.xh, q.yh);
        zx[l] = zx[l + 64] = make_float2(q.zh, q.xl);
        yz[l] = yz[l + 64] = make_float2(q.yl, q.zl);
        fxy[l] = fxy[l + 64] = make_float2(fx, fy);
        fz[l] = fz[l + 64] = make_float2(gz, q.zh + q.zh);
    }
    // r = target - source in FP32; zj = the source's height (its hi part),
    // zj2 = 2 zj
    __device__ __forceinline__ void diff(int e, const Pos2 &t, float &rx, float &ry, float &rz, float &fx, float &fy,
                                         float &gz, float &zj, float &zj2) const {
        using P = VOp<float>;
        const float2 a = xy[e], b = zx[e], c = yz[e], f = fxy[e], g = fz[e];
        rx = P::add(P::sub(t.xh, a.x), P::sub(t.xl, b.y));
        ry = P::add(P::sub(t.yh, a.y), P::sub(t.yl, c.x));
        rz = P::add(P::sub(t.zh, b.x), P::sub(t.zl, c.y));
        fx = f.x, fy = f.y, gz = g.x, zj = b.x, zj2 = g.y;
    }
};
template <>
// FP64 pairs: physical positions, so that the difference of two nearby
// positions is exact, scaled by 1/a afterwards (one rounding, relative);
// scaling the positions first would round each of them at the scale of its
// own coordinate, an error that grows as 1/a relative to the pair distance.
// zs: the source's height in units of a.
struct SymStage<double> {
    double x[128], y[128], z[128], zs[128], fx[128], fy[128], fz[128];
    __device__ __forceinline__ void put(int l, double px, double py, double pz, double gx, double gy, double gz,
                                        double pzs) {
        x[l] = x[l + 64] = px;
        y[l] = y[l + 64] = py;
        z[l] = z[l + 64] = pz;
        zs[l] = zs[l + 64] = pzs;
        fx[l] = fx[l + 64] = gx;
        fy[l] = fy[l + 64] = gy;
        fz[l] = fz[l + 64] = gz;
    }
    __device__ __forceinline__ void diff(int e, const Pos64 &t, double &rx, double &ry, double &rz, double &gx,
                                         double &gy, double &gz, double &zj, double &zj2) const {
        rx = (t.v[0] - x[e]) * t.ia, ry = (t.v[1] - y[e]) * t.ia, rz = (t.v[2] - z[e]) * t.ia;
        gx = fx[e], gy = fy[e], gz = fz[e];
        zj = zs[e];
        zj2 = zj + zj;
    }
};

// Target position in the form the stage's diff expects.
template <typename R>
struct TargetPos;
template <>
struct TargetPos<float> {
    using T = Pos2;
    static __device__ __forceinline__ T make(double x, double y, double z) {
        Pos2 p;
        p.set(x, y, z);
        return p;
    }
};
template <>
struct TargetPos<double> {
    using T = Pos64;
    static __device__ __forceinline__ T make(double x, double y, double z) { return Pos64{{x, y, z}, 1.0}; }
};

// One tile per wave.  B: block size (multiple of 64).
//
// Diagonal tiles (I == J) run the one-sided product over the block with the
// source read through the scalar cache.  Off-diagonal tiles form each
// unordered pair once: lane l of a 64-target sub-block meets source
// (l - s) mod 64 of a 64-source group at step s (read from LDS) and adds
// M_ij f_j to its target and M_ij^T f_i to an accumulator that travels with
// the source (rotated one lane per step).
template <typename SRC, int B, bool WALL>
__global__ __launch_bounds__(64) void pair_sym_kernel(const SymJob *__restrict__ jobs, int32_t n_jobs) {
    using R = typename SrcView<SRC>::R;
    constexpr int G = B / 64;
    __shared__ SymStage<R> st;
    const int64_t w = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= w) lo = mid; else hi = mid - 1;
    }
    const SymJob &J = jobs[lo];
    const int64_t slot = w - J.wg_begin;  // the tile's partials within its band
    int32_t I, Jb;
    tile_ij(J.t0 + slot, J.n_blk, &I, &Jb);
    const int64_t nb = J.nb;
    const int lane = threadIdx.x;
    // sources are read straight from the positions and forces (no packed
    // records): wave-uniform in the diagonal tiles (scalar cache), one per
    // lane when a group is staged
    const gptr<double> __restrict__ spos = (gptr<double>)J.tpos;
    const gptr<double> __restrict__ slam = (gptr<double>)J.lam;
    const bool diag = I == Jb;
    const int64_t s0 = (int64_t)Jb * B, s1 = min(s0 + B, nb);
    // lengths in units of the blob radius (see PairCoef): FP32 pairs scale
    // the positions (ps) before they are split into two floats, FP64 pairs
    // scale each difference (ds; see SymStage<double>)
    const double inv_a = 1.0 / J.a;
    const double ps = sizeof(R) == 4 ? inv_a : 1.0, ds = sizeof(R) == 4 ? 1.0 : inv_a;
    const R tiny = sizeof(R) == 4 ? (R)1e-30f : (R)1e-280;
    // tile sums: with FP32 pairs and B = 64 each one is an FP32 sum over 64
    // sources, stored exactly as a float; larger tiles add their groups of 64
    // in FP64 and store that sum as it is, so the FP32 part never spans more
    // than 64 sources
    using S = typename std::conditional<(B > 64), double, R>::type;
    const gmem<S> vout = as_global((S *)J.vpart + slot * (int64_t)B * 3);
    const gmem<S> uout = as_global((S *)J.upart + slot * (int64_t)B * 3);

    double u64[G][3];
#pragma unroll
    for (int g = 0; g < G; ++g) u64[g][0] = u64[g][1] = u64[g][2] = 0.0;

    for (int sub = 0; sub < G; ++sub) {
        const int64_t i = (int64_t)I * B + sub * 64 + lane;
        if ((int64_t)I * B + sub * 64 >= nb) break;  // wave-uniform
        const bool active = i < nb;
        const int64_t ii = active ? i : (int64_t)I * B + sub * 64;
        const double xi = as_global(J.tpos)[3 * ii] * ps, yi = as_global(J.tpos)[3 * ii + 1] * ps,
                     zi = as_global(J.tpos)[3 * ii + 2] * ps;
        auto tp = TargetPos<R>::make(xi, yi, zi);
        if constexpr (sizeof(R) == 8) tp.ia = ds;
        // the target's own force enters the transposed contraction
        const R fix = active ? (R)as_global(J.lam)[3 * ii] : (R)0, fiy = active ? (R)as_global(J.lam)[3 * ii + 1] : (R)0,
                fiz = active ? (R)as_global(J.lam)[3 * ii + 2] : (R)0;
        double vx = 0.0, vy = 0.0, vz = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t jb = s0 + 64 * g;
            if (jb >= s1) break;  // wave-uniform
            R ax = 0, ay = 0, az = 0;
            if (diag) {
                const int je = (int)min((int64_t)64, s1 - jb);
                for (int jj = 0; jj < je; ++jj) {
                    const int64_t j = jb + jj;
                    const double sx = spos[3 * j] * ps, sy = spos[3 * j + 1] * ps, sz = spos[3 * j + 2] * ps;
                    const R rx = (R)((xi - sx) * ds), ry = (R)((yi - sy) * ds), rz = (R)((zi - sz) * ds);
                    PairCoef<R, WALL> pc;
                    pc.eval(rx, ry, rz, (R)(sz * ds), tiny);
                    pc.template apply<false>(rx, ry, rz, (R)slam[3 * j], (R)slam[3 * j + 1], (R)slam[3 * j + 2], ax, ay,
                                             az);
                }
            } else {
                // stage the group (idle lanes carry a valid position with
                // zero force)
                const int64_t jl = jb + lane;
                const bool jvalid = jl < s1;
                const int64_t js = jvalid ? jl : jb;
                const double px = spos[3 * js] * ps, py = spos[3 * js + 1] * ps, pz = spos[3 * js + 2] * ps;
                const R gx = jvalid ? (R)slam[3 * js] : (R)0, gy = jvalid ? (R)slam[3 * js + 1] : (R)0,
                        gz = jvalid ? (R)slam[3 * js + 2] : (R)0;
                __syncthreads();  // the previous group's reads are done
                st.put(lane, px, py, pz, gx, gy, gz, pz * ds);
                __syncthreads();
                R ux = 0, uy = 0, uz = 0;
#pragma unroll 2
                for (int step = 0; step < 64; ++step) {
                    R rx, ry, rz, sfx, sfy, sfz, szj, szj2;
                    st.diff(lane - step + 64, tp, rx, ry, rz, sfx, sfy, sfz, szj, szj2);
                    PairCoef<R, WALL> pc;
                    const R rxy2 = VOp<R>::fma(ry, ry, VOp<R>::mul(rx, rx));
                    const R d2 = VOp<R>::fma(rz, rz, rxy2);
                    // overlapping pairs (r <= 2a) are rare away from the
                    // diagonal tiles: when no lane of the wave has one, the
                    // far branch alone is evaluated (wave-uniform branch)
                    if (__ballot(d2 <= (R)4) != 0)
                        pc.template eval_d2<true>(rxy2, d2, rz, szj, szj2, tiny);
                    else
                        pc.template eval_d2<false>(rxy2, d2, rz, szj, szj2, tiny);
                    pc.template apply<false>(rx, ry, rz, sfx, sfy, sfz, ax, ay, az);
                    pc.template apply<true>(rx, ry, rz, fix, fiy, fiz, ux, uy, uz);
                    ux = rot1(ux), uy = rot1(uy), uz = rot1(uz);
                }
                // after 64 rotations each accumulator is back on its source's lane
                u64[g][0] += (double)ux;
                u64[g][1] += (double)uy;
                u64[g][2] += (double)uz;
            }
            vx += (double)ax;
            vy += (double)ay;
            vz += (double)az;
        }
        if (active) {
            const int e = sub * 64 + lane;
            vout[e] = (S)vx;
            vout[B + e] = (S)vy;
            vout[2 * B + e] = (S)vz;
        }
    }
    if (!diag) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t j = s0 + 64 * g + lane;
            if (j < s1) {
                const int e = 64 * g + lane;
                uout[e] = (S)u64[g][0];
                uout[B + e] = (S)u64[g][1];
                uout[2 * B + e] = (S)u64[g][2];
            }
        }
    }
}

// One-sided FP32 product (targets and sources may differ: small systems and
// the flow field).  A workgroup of 256 lanes owns 256 targets and one chunk of
// sources; the sources are staged in LDS 256 at a time, as two-float
// positions, and every wave then visits them one by one with the same
// address on all lanes (LDS broadcast), so the pair arithmetic runs on
// registers in VOP3 form.  Sums are FP32 over aligned blocks of 64 sources
// and FP64 across blocks, as in the symmetric product.
struct SrcStage {
    float2 xy[kPairBlock], zx[kPairBlock], yz[kPairBlock], fxy[kPairBlock], fz[kPairBlock];
};

template <bool WALL>
__global__ __launch_bounds__(kPairBlock) void pair_lds_f32_kernel(const PairJob *__restrict__ jobs, int32_t n_jobs) {
    using P = VOp<float>;
    __shared__ SrcStage st;
    const int64_t w = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_begin <= w) lo = mid; else hi = mid - 1;
    }
    const PairJob &J = jobs[lo];
    const int64_t lt = w - J.tile_begin;
    const int32_t split = (int32_t)(lt / J.n_tblock);
    const int64_t t0 = (lt % J.n_tblock) * kPairBlock;
    const int64_t s0 = split * J.chunk;
    const int64_t s1 = min(s0 + J.chunk, J.ns);
    const int tid = threadIdx.x;
    const int64_t i = t0 + tid;
    const bool active = i < J.nb;
    const int64_t ii = active ? i : t0;  // idle lanes shadow a valid target
    const gmem<const double> tpos = as_global(J.tpos);
    // positions in units of the blob radius (see PairCoef)
    const double inv_a = 1.0 / J.a;
    Pos2 tp;
    tp.set(tpos[3 * ii] * inv_a, tpos[3 * ii + 1] * inv_a, tpos[3 * ii + 2] * inv_a);
    const gmem<const SrcF32> src = as_global((const SrcF32 *)J.src);
    const float tiny = 1e-30f;
    double vx = 0.0, vy = 0.0, vz = 0.0;

    for (int64_t jb = s0; jb < s1; jb += kPairBlock) {
        const int64_t j = jb + tid;
        const int64_t js = j < s1 ? j : jb;
        const gmem<const SrcF32> r = src + js;
        Pos2 q;
        q.set(r->x * inv_a, r->y * inv_a, r->z * inv_a);
        const float fx = j < s1 ? r->fx : 0.f, fy = j < s1 ? r->fy : 0.f, gz = j < s1 ? r->fz : 0.f;
        __syncthreads();  // the previous block's reads are done
        st.xy[tid] = make_float2(q.xh, q.yh);
        st.zx[tid] = make_float2(q.zh, q.xl);
        st.yz[tid] = make_float2(q.yl, q.zl);
        st.fxy[tid] = make_float2(fx, fy);
        st.fz[tid] = make_float2(gz, q.zh + q.zh);
        __syncthreads();
        const int ne = (int)min((int64_t)kPairBlock, s1 - jb);
        for (int g = 0; g < ne; g += kAccBlock) {
            const int ge = min(kAccBlock, ne - g);
            float ax = 0.f, ay = 0.f, az = 0.f;
            for (int k = 0; k < ge; ++k) {
                const int e = g + k;
                const float2 xy = st.xy[e], zx = st.zx[e], yz = st.yz[e], f = st.fxy[e], fzz = st.fz[e];
                const float rx = P::add(P::sub(tp.xh, xy.x), P::sub(tp.xl, zx.y));
                const float ry = P::add(P::sub(tp.yh, xy.y), P::sub(tp.yl, yz.x));
                const float rz = P::add(P::sub(tp.zh, zx.x), P::sub(tp.zl, yz.y));
                const float rxy2 = P::fma(ry, ry, P::mul(rx, rx));
                const float d2 = P::fma(rz, rz, rxy2);
                PairCoef<float, WALL> pc;
                if (__ballot(d2 <= 4.f) != 0)
                    pc.template eval_d2<true>(rxy2, d2, rz, zx.x, fzz.y, tiny);
                else
                    pc.template eval_d2<false>(rxy2, d2, rz, zx.x, fzz.y, tiny);
                pc.template apply<false>(rx, ry, rz, f.x, f.y, fzz.x, ax, ay, az);
            }
            vx += (double)ax;
            vy += (double)ay;
            vz += (double)az;
        }
    }
    if (active) {
        const gmem<double> out = as_global(J.partial + ((int64_t)split * J.nb + i) * 3);
        out[0] = vx;
        out[1] = vy;
        out[2] = vz;
    }
}

hipError_t launch_pair_lds_f32(bool wall, const PairJob *jobs, int32_t n_jobs, int64_t n_tiles, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    dim3 g((unsigned)n_tiles), b(kPairBlock);
    if (wall)
        hipLaunchKernelGGL(pair_lds_f32_kernel<true>, g, b, 0, s, jobs, n_jobs);
    else
        hipLaunchKernelGGL(pair_lds_f32_kernel<false>, g, b, 0, s, jobs, n_jobs);
    return hipGetLastError();
}

// v[k] = pref * (sum_{J >= K} vpart[tile(K,J)][kk] + sum_{I < K} upart[tile(I,K)][kk]),
// taken band by band.  Within a band the contributions of a blob of block K
// are listed as its row tiles (K, J >= K) when K is one of the band's rows,
// then its column tiles (I, K) for the band's rows I < K; the first band's
// sum is stored in an FP64 accumulator, later bands add theirs to it, and
// the last band writes pref times the total (one band: no accumulator, the
// sum goes straight to the output).
constexpr int kRedWaves = 16;

// One workgroup of 16 waves per 64 blobs of a block: wave q adds the blobs'
// contributions q, q + 16, ... in the order above, each read as one row of 64
// consecutive values per component of the [tile][3][B] partials; the waves'
// sums are then added in a fixed order.  Workgroups past n_red carry the
// saddle body rows of a solve step (16 bodies per workgroup, a wave each):
// they read only the Krylov vector, so they share the launch with the
// reduction instead of taking one of their own.
__global__ __launch_bounds__(1024) void sym_reduce_kernel(const SymJob *__restrict__ jobs, int32_t n_jobs,
                                                          int64_t n_red, const SaddleJob *__restrict__ sd,
                                                          int32_t n_sd, int64_t n_body) {
    __shared__ double part[kRedWaves][3][64];
    const int64_t w = blockIdx.x;
    const int q = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (w >= n_red) {
        const int64_t body = (w - n_red) * kRedWaves + q;
        if (body < n_body) saddle_body_rows(sd, n_sd, body, lane);
        return;
    }
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].red_begin <= w) lo = mid; else hi = mid - 1;
    }
    const SymJob &J = jobs[lo];
    const int32_t B = J.B, T = J.n_blk, I0 = J.I0, I1 = J.I1;
    // groups of 64 never straddle a block (B is a multiple of 64); the last
    // band covers every blob, the others the blobs of blocks >= I0
    const int64_t k0 = (J.last ? 0 : (int64_t)I0 * B) + (w - J.red_begin) * 64;
    const int64_t k = k0 + lane;
    const int32_t K = (int32_t)(k0 / B);
    const int64_t kk = k0 % B + lane;
    double s[3] = {0.0, 0.0, 0.0};
    if (k < J.nb && K >= I0) {
        auto slot = [&](int64_t i, int64_t j) { return i * T - i * (i - 1) / 2 + (j - i) - J.t0; };
        const int32_t nv = K < I1 ? T - K : 0;            // row tiles (K, K + c)
        const int32_t n = nv + (K < I1 ? K : I1) - I0;    // then column tiles (I0 + c - nv, K)
        if (J.f32 && B == 64) {  // float partials (see the tile kernel)
#pragma unroll 4
            for (int32_t c = q; c < n; c += kRedWaves) {
                const gmem<const float> p = as_global(c < nv ? (const float *)J.vpart + slot(K, K + c) * B * 3 + kk
                                                             : (const float *)J.upart + slot(I0 + c - nv, K) * B * 3 + kk);
                s[0] += (double)p[0], s[1] += (double)p[B], s[2] += (double)p[2 * B];
            }
        } else {
#pragma unroll 4
            for (int32_t c = q; c < n; c += kRedWaves) {
                const gmem<const double> p = as_global(c < nv ? J.vpart + slot(K, K + c) * B * 3 + kk
                                                              : J.upart + slot(I0 + c - nv, K) * B * 3 + kk);
                s[0] += p[0], s[1] += p[B], s[2] += p[2 * B];
            }
        }
    }
    part[q][0][lane] = s[0], part[q][1][lane] = s[1], part[q][2][lane] = s[2];
    __syncthreads();
    if (q == 0 && k < J.nb) {
        double t[3] = {0.0, 0.0, 0.0};
        if (!J.first) {
            const gmem<const double> a = as_global((const double *)J.acc + 3 * k);
            t[0] = a[0], t[1] = a[1], t[2] = a[2];
        }
        for (int r = 0; r < kRedWaves; ++r) t[0] += part[r][0][lane], t[1] += part[r][1][lane], t[2] += part[r][2][lane];
        if (!J.last) {
            const gmem<double> a = as_global(J.acc + 3 * k);
            a[0] = t[0], a[1] = t[1], a[2] = t[2];
            return;
        }
        const double v[3] = {J.pref * t[0], J.pref * t[1], J.pref * t[2]};
        if (J.epi) {
            // inside a solve: the blob rows of the saddle-point operator
            saddle_blob_row(*(const SaddleJob *)J.epi, k, v);
        } else {
            const gmem<double> o = as_global(J.vel + 3 * k);
            o[0] = v[0];
            o[1] = v[1];
            o[2] = v[2];
        }
    }
}

void sym_plan(int64_t nb, int32_t *B, int32_t *n_blk) {
    int32_t b = nb <= 16384 ? 64 : nb <= 65536 ? 128 : 256;
    *B = b;
    *n_blk = (int32_t)((nb + b - 1) / b);
}

int64_t sym_tiles(int64_t nb) {
    int32_t B, T;
    sym_plan(nb, &B, &T);
    return (int64_t)T * (T + 1) / 2;
}

std::vector<SymBand> sym_bands(int64_t nb, size_t band_bytes) {
    int32_t B, T;
    sym_plan(nb, &B, &T);
    const int64_t cap = std::max<int64_t>(1, (int64_t)(band_bytes / ((size_t)B * 3 * 2 * sizeof(double))));
    std::vector<SymBand> out;
    int64_t t = 0;
    int32_t I = 0;
    while (I < T) {
        SymBand b{I, I, t, 0};
        while (b.I1 < T && (b.I1 == I || b.tiles + (T - b.I1) <= cap)) b.tiles += T - b.I1, ++b.I1;
        t += b.tiles;
        I = b.I1;
        out.push_back(b);
    }
    return out;
}

size_t sym_band_partial_doubles(int64_t nb, size_t band_bytes) {
    int32_t B, T;
    sym_plan(nb, &B, &T);
    int64_t most = 0;
    for (const SymBand &b : sym_bands(nb, band_bytes)) most = std::max(most, b.tiles);
    return (size_t)most * B * 3 * 2;  // vpart + upart
}

int64_t sym_reduce_groups_band(int64_t nb, int32_t B, const SymBand &b, bool last) {
    const int64_t first = last ? 0 : (int64_t)b.I0 * B;
    return (nb - first + 63) / 64;
}

template <typename SRC, bool WALL>
static void launch_sym_b(int B, const SymJob *jobs, int32_t n_jobs, int64_t n_tiles, hipStream_t s) {
    dim3 g((unsigned)n_tiles), b(64);
    switch (B) {
        case 64: hipLaunchKernelGGL((pair_sym_kernel<SRC, 64, WALL>), g, b, 0, s, jobs, n_jobs); break;
        case 128: hipLaunchKernelGGL((pair_sym_kernel<SRC, 128, WALL>), g, b, 0, s, jobs, n_jobs); break;
        default: hipLaunchKernelGGL((pair_sym_kernel<SRC, 256, WALL>), g, b, 0, s, jobs, n_jobs); break;
    }
}

hipError_t launch_pair_sym(int precision, bool wall, int B, const SymJob *jobs, int32_t n_jobs, int64_t n_tiles,
                           hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    if (precision == RMB_PREC_FP32_PAIRS) {
        if (wall) launch_sym_b<SrcF32, true>(B, jobs, n_jobs, n_tiles, s);
        else launch_sym_b<SrcF32, false>(B, jobs, n_jobs, n_tiles, s);
    } else {
        if (wall) launch_sym_b<SrcF64, true>(B, jobs, n_jobs, n_tiles, s);
        else launch_sym_b<SrcF64, false>(B, jobs, n_jobs, n_tiles, s);
    }
    return hipGetLastError();
}

// Job records written by a one-thread kernel from its argument (no host
// staging buffer): used where a caller's stream must not depend on host
// memory the library would have to allocate.
template <typename T>
__device__ __forceinline__ void store_words(const T &j, T *dst) {
    static_assert(sizeof(T) % 4 == 0, "job records are whole words");
    const int *w = (const int *)&j;
    const gmem<int> d = as_global((int *)dst);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) d[k] = w[k];
}
__global__ void store_sym_job_kernel(SymJob j, SymJob *dst) { store_words(j, dst); }
__global__ void store_pair_job_kernel(PairJob j, PairJob *dst) { store_words(j, dst); }

hipError_t launch_store_sym_job(const SymJob &j, SymJob *dst, hipStream_t s) {
    hipLaunchKernelGGL(store_sym_job_kernel, dim3(1), dim3(1), 0, s, j, dst);
    return hipGetLastError();
}
hipError_t launch_store_pair_job(const PairJob &j, PairJob *dst, hipStream_t s) {
    hipLaunchKernelGGL(store_pair_job_kernel, dim3(1), dim3(1), 0, s, j, dst);
    return hipGetLastError();
}

hipError_t launch_sym_reduce(const SymJob *jobs, int32_t n_jobs, int64_t n_wg, const SaddleJob *sd, int32_t n_sd,
                             int64_t n_body, hipStream_t s) {
    if (!sd || n_sd <= 0) n_body = 0;
    const int64_t total = n_wg + (n_body + kRedWaves - 1) / kRedWaves;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(sym_reduce_kernel, dim3((unsigned)total), dim3(64 * kRedWaves), 0, s, jobs, n_jobs, n_wg, sd,
                       n_sd, n_body);
    return hipGetLastError();
}

}  // namespace rmb

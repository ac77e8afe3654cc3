// Per-body and Krylov kernel interfaces (internal).
#pragma once

#include "rmb_common.h"

namespace rmb {

// Largest 3n x 3n block handled by the LDS-resident per-body path.
constexpr int kSmallBodyMaxM = 84;  // 28 blobs: build workspace (m^2 + 13m + 36 doubles) stays under 64 KiB of LDS

// One body of one system, for preconditioner build and apply.
struct BodyWork {
    const double *pos;  // system's blob positions [nb][3]
    const double *q;    // this body's tracking point (3 doubles)
    double *factor;     // LDS path: Li = L^-1 (col-major), Y (m x 6), S^-1 (6 x 6);
                        // large path: L (padded, col-major), Y, diagonal-block
                        // inverses of L, Sc (Cholesky of S)
    int64_t blob0;      // first blob of the body
    int32_t n_blobs;
    int32_t body;       // body index within its system
    int32_t wall;
    int32_t pad;
    double a, pref;     // blob radius, 1/(6 pi eta a)
    int *flag;          // build status of the body's system (bits 4: not SPD, 8: singular)
    const double *shift;  // build only: the system's permeability shifts d (indexed by blob) or NULL
    const double *rot;  // apply only: NULL, or the body's rotation R (3 x 3, row-major) when the
                        // factor is that of a shared reference shape; the body's block is then
                        // R~ P_ref^-1 R~^T (R~ = R on every 3-vector)
};

// A body whose block exceeds the LDS path: padded to Mp (multiple of 32).
struct BigBody {
    BodyWork w;
    int32_t Mp;
    int32_t pad;
};

inline bool is_large_body(int64_t n_blobs) { return 3 * n_blobs > kSmallBodyMaxM; }
// Large bodies: the block with 6 bordered rows (K_p^T), rounded up to the
// 64-column panels of the factorisation.
inline int64_t padded_dim(int64_t n_blobs) { return (3 * n_blobs + 6 + 63) / 64 * 64; }

// Factor storage of one body (doubles).  Small bodies: L^-1 (lower
// triangle, packed by columns: column c holds rows c..m-1 from
// packed_col(m, c)), Y (m x 6), S^-1 (6 x 6).  Large bodies, padded
// dimension Mp: L (Mp x Mp), Y (Mp x 6), inverses of L's diagonal blocks
// (Mp x 32), Sc (6 x 6).
__host__ __device__ inline int64_t packed_col(int64_t m, int64_t c) { return c * m - c * (c - 1) / 2; }
inline int64_t factor_doubles(int64_t n_blobs) {
    if (!is_large_body(n_blobs)) {
        const int64_t m = 3 * n_blobs;
        return m * (m + 1) / 2 + 6 * m + 36;
    }
    const int64_t Mp = padded_dim(n_blobs);
    return Mp * Mp + 6 * Mp + 32 * Mp + 36;
}

// P^-1 applied to `nrhs` saddle vectors of one system (vector r at in + r*ld).
// mode 1 (resistance problem): the vectors hold blob forces only and the
// apply is lambda_p = M_pp^-1 s_p per body, with the same factors.
struct PrecondApplyJob {
    const BodyWork *items;  // the system's bodies (BigBody records for the large-body kernel)
    const double *in;
    double *out;
    int64_t ld;             // stride between right-hand sides
    int64_t nb3;            // 3 * n_blobs (offset of the U block)
    int64_t wg_begin;       // first workgroup of this system in the launch
    int32_t n_items;
    int32_t nrhs;
    int32_t mode;
    int32_t pad;
};

// Saddle-point operator rows around a finished pair product.
struct SaddleJob {
    const double *pos;
    const double *q;
    const int64_t *body_off;  // device [N+1]
    const int32_t *blob_body; // device [nb]
    const double *partial;    // [n_split][nb][3] pair sums
    const double *x;          // input [lambda; U] (only U read for blob rows, lambda for body rows)
    const double *b;          // NULL: y = A x; else y = b - A x
    const double *shift;      // permeability shifts d [nb] (M + diag(d)) or NULL
    double *y;
    int64_t nb;
    int64_t blk_begin;        // first blob-row workgroup of this system
    int64_t body_begin;       // first body-row workgroup of this system
    int32_t n_split;
    int32_t resist;           // 1: resistance operator y = (M + diag(d)) lambda, no K terms or body rows
    double pref;
};

// Blob row i of the saddle-point operator from the finished product v_i
// (prefactor applied): y_i = v_i + d_i x_i - (u_p + omega_p x (r_i - q_p)), or
// b_i - y_i; the resistance form drops the rigid-motion term.
__device__ __forceinline__ void saddle_blob_row(const SaddleJob &J, int64_t i, const double v[3]) {
    const int64_t n3 = 3 * J.nb;
    double ku[3] = {0.0, 0.0, 0.0};
    if (!J.resist) {
        const int p = as_global(J.blob_body)[i];
        const gmem<const double> U = as_global(J.x + n3 + 6 * (int64_t)p);
        const gmem<const double> q = as_global(J.q + 3 * (int64_t)p);
        const double d[3] = {as_global(J.pos)[3 * i] - q[0], as_global(J.pos)[3 * i + 1] - q[1],
                             as_global(J.pos)[3 * i + 2] - q[2]};
        ku[0] = U[0] + U[4] * d[2] - U[5] * d[1];
        ku[1] = U[1] + U[5] * d[0] - U[3] * d[2];
        ku[2] = U[2] + U[3] * d[1] - U[4] * d[0];
    }
    const double shift = J.shift ? as_global(J.shift)[i] : 0.0;
    for (int c = 0; c < 3; ++c) {
        const double y = v[c] + shift * as_global(J.x)[3 * i + c] - ku[c];
        as_global(J.y)[3 * i + c] = J.b ? as_global(J.b)[3 * i + c] - y : y;
    }
}

// Body rows of the saddle-point operator for body w of the job list (its
// global index over all jobs' bodies), one 64-lane wave: -K^T x, or
// b_body + K^T x with a right-hand side.  `lane` is the wave lane 0..63.
__device__ __forceinline__ void saddle_body_rows(const SaddleJob *__restrict__ jobs, int32_t n_jobs, int64_t w,
                                                 int lane) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].body_begin <= w) lo = mid; else hi = mid - 1;
    }
    const SaddleJob &J = jobs[lo];
    const int64_t p = w - J.body_begin;
    const int64_t b0 = as_global(J.body_off)[p], b1 = as_global(J.body_off)[p + 1];
    const gmem<const double> q = as_global(J.q + 3 * p);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = b0 + lane; i < b1; i += 64) {
        const double l[3] = {as_global(J.x)[3 * i], as_global(J.x)[3 * i + 1], as_global(J.x)[3 * i + 2]};
        const double d[3] = {as_global(J.pos)[3 * i] - q[0], as_global(J.pos)[3 * i + 1] - q[1],
                             as_global(J.pos)[3 * i + 2] - q[2]};
        acc[0] += l[0];
        acc[1] += l[1];
        acc[2] += l[2];
        acc[3] += d[1] * l[2] - d[2] * l[1];
        acc[4] += d[2] * l[0] - d[0] * l[2];
        acc[5] += d[0] * l[1] - d[1] * l[0];
    }
    for (int k = 0; k < 6; ++k) {
        double v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[k] = v;
    }
    if (lane == 0) {
        const int64_t o = 3 * J.nb + 6 * p;
        for (int k = 0; k < 6; ++k) as_global(J.y)[o + k] = J.b ? as_global(J.b)[o + k] + acc[k] : -acc[k];
    }
}

hipError_t launch_precond_build_small(const BodyWork *items, int32_t n_items, int max_m, hipStream_t s);
hipError_t launch_precond_apply_small(const PrecondApplyJob *jobs, int32_t n_jobs, int64_t n_wg,
                                      int32_t max_rhs, int max_m, hipStream_t s);
// Large bodies: assembly, MFMA left-looking Cholesky, projection; and the
// apply (<= 8 rhs per workgroup).  `variant` selects one of
// large_variant_count() tile shapes (panel width, row tiles per wave,
// staged columns); every shape stores the same factor layout, so the apply
// does not depend on the shape.
int large_variant_count();
void large_variant_shape(int variant, int *panel, int *row_tiles, int *chunk);
hipError_t launch_precond_build_large(const BigBody *items, int32_t n_items, int max_Mp, int variant, hipStream_t s);
hipError_t launch_precond_apply_large(const PrecondApplyJob *jobs, int32_t n_jobs, int64_t n_wg, int32_t max_rhs,
                                      int max_Mp, hipStream_t s);
// Resistance problem (eq:resistance_problem): b_i = u_p + omega_p x (r_i - q_p)
// + slip_i for blob i of body p (U device [N][6], slip [nb][3] or NULL).
hipError_t launch_build_rhs_resist(const double *U, const double *slip, const double *pos, const double *q,
                                   const int32_t *blob_body, int64_t nb, double *b, hipStream_t s);
// F_p = K_p^T lambda = (sum_i lambda_i, sum_i (r_i - q_p) x lambda_i), [N][6].
hipError_t launch_body_forces(const double *pos, const double *q, const int64_t *body_off, const double *lam,
                              int64_t N, double *F, hipStream_t s);

// Rotation matrices (row-major, 9 doubles per body) of N quaternions
// (w, x, y, z), normalised on the fly; a zero or non-finite quaternion sets
// bit 16 of *flag and yields the identity.
hipError_t launch_quat_rotations(const double *quat, int64_t N, double *rot, int *flag, hipStream_t s);

hipError_t launch_saddle(const SaddleJob *jobs, int32_t n_jobs, int64_t n_blob_blocks, int64_t n_bodies,
                         hipStream_t s);

// ---------------------------------------------------------------------------
// Krylov vector kernels
// ---------------------------------------------------------------------------

constexpr int kSeg = 512;     // vector elements per chunk (256 threads x 2)
constexpr int kMaxSeg = 256;  // most workgroups per system in a Krylov launch

// Workgroups and chunks per workgroup covering an n-vector (n_seg <= kMaxSeg).
inline void krylov_segments(int64_t n, int32_t *n_seg, int32_t *n_chunk) {
    const int64_t chunks = (n + kSeg - 1) / kSeg;
    const int64_t per = (chunks + kMaxSeg - 1) / kMaxSeg;
    *n_chunk = (int32_t)(per > 0 ? per : 1);
    *n_seg = (int32_t)((n + (int64_t)*n_chunk * kSeg - 1) / ((int64_t)*n_chunk * kSeg));
}

struct KrylovJob {
    double *V;          // basis vectors, vector k at V + k*ldv
    int64_t ldv;
    double *w;          // vector being orthogonalised / normalised / combined into
    double *vnext;      // normalised output (V + kk*ldv)
    double *P1, *P2;    // partial dots [(kmax+1) x n_seg]
    double *P3;         // partial squared norms [n_seg]
    double *hcol;       // output: h[0..kk-1] then the norm at hcol[kk]
    double *hred;       // h1 [256], kept between the second and third pass
    const double *coef; // combine coefficients (kk of them)
    double *x;          // axpy target
    const double *t;    // axpy source
    int64_t n;
    int64_t wg_begin;
    int32_t n_seg;      // workgroups of this system
    int32_t n_chunk;    // 512-element chunks per workgroup
    int32_t kk;
    int64_t u0;         // velocity norms: first element of the body part of x and t
};

// CGS2 orthogonalisation of w against V[0..kk-1] and normalisation into
// vnext, writing hcol; kk = 0 normalises w alone.  Four launches.
hipError_t launch_orthogonalise(const KrylovJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s);
// w = sum_{k<kk} coef[k] V[k]
hipError_t launch_combine(const KrylovJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s);
// x += t
hipError_t launch_axpy(const KrylovJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s);
// One workgroup per job (wg_begin = its index): hcol[1] = sum of t[e]^2 and
// hcol[2] = sum of x[e]^2 over e in [u0, n), summed in a fixed order.
hipError_t launch_unorm(const KrylovJob *jobs, int32_t n_jobs, hipStream_t s);

// ---------------------------------------------------------------------------
// misc per-system kernels
// ---------------------------------------------------------------------------

// b = [slip or 0 ; -F]
hipError_t launch_build_rhs(const double *FT, const double *slip, int64_t nb, int64_t N, double *b,
                            hipStream_t s);
// blob_body[i] = p for i in [off[p], off[p+1])
hipError_t launch_blob_body(const int64_t *off, int64_t N, int32_t *blob_body, hipStream_t s);

}  // namespace rmb

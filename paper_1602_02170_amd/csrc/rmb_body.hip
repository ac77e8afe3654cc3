// Per-body kernels: rigid kinematics K, K^T (eq:noslip_rigid,
// eq:rigidSystem), the saddle-point operator's assembly (eq:saddle_M), and
// the indefinite block-diagonal preconditioner (eq:M_tilde_block_diag,
// eq:indef_block_P, eq:saddle_M_precon) for bodies small enough that a
// body's 3n x 3n mobility block fits in LDS.
//
// Preconditioner of body p (m = 3 n_p):
//   M_pp = L L^T,  Y = L^-1 K_p (m x 6),  S = Y^T Y = K_p^T M_pp^-1 K_p
// and for a right-hand side (s_p, bottom_p) with F_p = -bottom_p:
//   t = L^-1 s,  U = S^-1 (F - Y^T t),  lambda = L^-T (t + Y U).
// Bodies on the LDS path store Li = L^-1 (lower triangle packed by columns),
// Y (row-major) and S^-1, so that an apply is two triangular matrix-vector
// products.
#include <cmath>

#include "rmb_blocks.h"
#include "rmb_body.h"

namespace rmb {

// ---------------------------------------------------------------------------
// small-body preconditioner: build
// ---------------------------------------------------------------------------

// One workgroup (one wave) per body; the body's block lives in LDS.
__global__ __launch_bounds__(64) void precond_build_small_kernel(const BodyWork *__restrict__ items,
                                                                 int32_t n_items) {
    extern __shared__ double lds[];
    const BodyWork it = items[blockIdx.x];
    const int n = it.n_blobs, m = 3 * n, tid = threadIdx.x;
    double *A = lds;              // m x m, row-major
    double *Y = A + m * m;        // m x 6
    double *S = Y + 6 * m;        // 6 x 6
    double *Ld = S + 36;          // L's diagonal (m)
    double *Kp = Ld + m;          // K_p (m x 6, row-major)
    __shared__ int bad;
    if (tid == 0) bad = 0;

    // 1. assemble M_pp (with prefactor)
    for (int pq = tid; pq < n * n; pq += blockDim.x) {
        const int i = pq / n, j = pq % n;
        const gmem<const double> ri = as_global(it.pos + 3 * (int64_t)(it.blob0 + i));
        const gmem<const double> rj = as_global(it.pos + 3 * (int64_t)(it.blob0 + j));
        double B[9];
        const double a_i[3] = {ri[0], ri[1], ri[2]}, a_j[3] = {rj[0], rj[1], rj[2]};
        pair_block_f64(a_i, a_j, it.a, it.wall != 0, B);
        // permeable bodies: d_i on the diagonal (eq:permeable_slip)
        const double d = (i == j && it.shift) ? as_global(it.shift)[it.blob0 + i] : 0.0;
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q)
                A[(3 * i + p) * m + 3 * j + q] = it.pref * B[3 * p + q] + (p == q ? d : 0.0);
    }
    __syncthreads();

    // 2. right-looking Cholesky, lower triangle, in place, one barrier per
    //    column: the trailing update takes column j unscaled with the pivot
    //    d_jj (a_ik -= a_ij a_kj / d_jj), since no later column reads it,
    //    and all columns are scaled by 1/sqrt(d_jj) in one pass at the end
    //    (Ld holds the pivots meanwhile).
    for (int j = 0; j < m; ++j) {
        const double dj0 = A[j * m + j];
        const double dj = dj0 > 0.0 ? dj0 : 1.0;
        if (tid == 0) {
            if (!(dj0 > 0.0)) bad = 1;
            Ld[j] = dj;
        }
        const double inv_d = 1.0 / dj;
        // lanes as an 8 x 8 grid over the trailing lower triangle (no index
        // division): lane (a, b) takes row I0 + a and columns K0 + b and
        // K0 + 8 + b, loads before stores
        const int a = tid >> 3, b = tid & 7;
        for (int I0 = j + 1; I0 < m; I0 += 8) {
            const int i = I0 + a;
            const bool iv = i < m;
            const double aij = iv ? A[i * m + j] * inv_d : 0.0;
            for (int K0 = j + 1; K0 <= I0; K0 += 16) {
                const int k0 = K0 + b, k1 = K0 + 8 + b;
                const bool u0 = iv && k0 <= i, u1 = iv && k1 <= i;
                const double x0 = u0 ? A[i * m + k0] - aij * A[k0 * m + j] : 0.0;
                const double x1 = u1 ? A[i * m + k1] - aij * A[k1 * m + j] : 0.0;
                if (u0) A[i * m + k0] = x0;
                if (u1) A[i * m + k1] = x1;
            }
        }
        __syncthreads();
    }
    for (int c = tid; c < m; c += blockDim.x) {
        const double l = sqrt(Ld[c]);
        Ld[c] = l;
        Y[c] = 1.0 / l;  // Y is free until step 4
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += blockDim.x) {
        const int i = e / m, c = e - i * m;  // row-major A[i][c]
        if (c < i) A[e] *= Y[c];
        else if (c == i) A[e] = Ld[c];
    }
    __syncthreads();

    // 3. Li = L^-1, column-major in A.  Lane c forms column c below the
    //    diagonal into A's upper triangle (A[c m + r], r > c), reading L from
    //    the lower triangle, which no lane writes; the diagonal follows once
    //    every column is done (entries above Li's diagonal are never read).
    gmem<double> out = as_global(it.factor);
    const gmem<const double> q = as_global(it.q);
    for (int c = tid; c < m; c += blockDim.x) Ld[c] = A[c * m + c];
    __syncthreads();
    for (int c = tid; c < m; c += blockDim.x) {
        const double lcc = 1.0 / Ld[c];
        for (int r = c + 1; r < m; ++r) {
            // four independent partial sums: the loads and FMAs of a row
            // overlap instead of forming one dependent chain
            double p[4] = {A[r * m + c] * lcc, 0.0, 0.0, 0.0};
            int k = c + 1;
            for (; k + 3 < r; k += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) p[u] += A[r * m + k + u] * A[c * m + k + u];
            }
            for (; k < r; ++k) p[0] += A[r * m + k] * A[c * m + k];
            A[c * m + r] = -((p[0] + p[1]) + (p[2] + p[3])) / Ld[r];
        }
    }
    __syncthreads();
    for (int c = tid; c < m; c += blockDim.x) A[c * m + c] = 1.0 / Ld[c];
    __syncthreads();
    // 4. Y = Li K_p (K_p staged first), S = Y^T Y
    for (int e = tid; e < 6 * m; e += blockDim.x) {
        const int c = e / 6, k = e % 6, i = c / 3;
        const gmem<const double> ri = as_global(it.pos + 3 * (int64_t)(it.blob0 + i));
        const double d[3] = {ri[0] - q[0], ri[1] - q[1], ri[2] - q[2]};
        Kp[e] = K_entry(d, c % 3, k);
    }
    __syncthreads();
    for (int e = tid; e < 6 * m; e += blockDim.x) {
        const int row = e / 6, k = e % 6;
        double p[4] = {0.0, 0.0, 0.0, 0.0};
        int c = 0;
        for (; c + 3 <= row; c += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) p[u] += A[(c + u) * m + row] * Kp[(c + u) * 6 + k];
        }
        for (; c <= row; ++c) p[0] += A[c * m + row] * Kp[c * 6 + k];
        Y[row * 6 + k] = (p[0] + p[1]) + (p[2] + p[3]);
    }
    __syncthreads();
    if (tid < 36) {
        const int r = tid / 6, c = tid % 6;
        double acc = 0.0;
        for (int l = 0; l < m; ++l) acc += Y[l * 6 + r] * Y[l * 6 + c];
        S[tid] = acc;
    }
    __syncthreads();
    // 5. S^-1 through its Cholesky factor (one lane)
    if (tid == 0) {
        double Lc[36], Inv[36];
        for (int j = 0; j < 6; ++j) {
            double dj = S[j * 6 + j];
            for (int k = 0; k < j; ++k) dj -= Lc[j * 6 + k] * Lc[j * 6 + k];
            if (!(dj > 0.0)) {
                bad |= 2;
                dj = 1.0;
            }
            const double ljj = sqrt(dj);
            Lc[j * 6 + j] = ljj;
            for (int i = j + 1; i < 6; ++i) {
                double v = S[i * 6 + j];
                for (int k = 0; k < j; ++k) v -= Lc[i * 6 + k] * Lc[j * 6 + k];
                Lc[i * 6 + j] = v / ljj;
            }
        }
        for (int col = 0; col < 6; ++col) {  // S^-1 e_col = Lc^-T Lc^-1 e_col
            double u[6];
            for (int i = 0; i < 6; ++i) {
                double v = i == col ? 1.0 : 0.0;
                for (int k = 0; k < i; ++k) v -= Lc[i * 6 + k] * u[k];
                u[i] = v / Lc[i * 6 + i];
            }
            for (int i = 5; i >= 0; --i) {
                double v = u[i];
                for (int k = i + 1; k < 6; ++k) v -= Lc[k * 6 + i] * Inv[k * 6 + col];
                Inv[i * 6 + col] = v / Lc[i * 6 + i];
            }
        }
        for (int e = 0; e < 36; ++e) S[e] = Inv[e];
    }
    __syncthreads();

    // 6. store Li (lower triangle packed by columns), Y, S^-1
    const int np = m * (m + 1) / 2;
    for (int e = tid; e < m * m; e += blockDim.x) {
        const int c = e / m, r = e - c * m;
        if (r >= c) out[packed_col(m, c) + r - c] = A[e];
    }
    for (int e = tid; e < 6 * m; e += blockDim.x) out[np + e] = Y[e];
    for (int e = tid; e < 36; e += blockDim.x) out[np + 6 * m + e] = S[e];
    // bit 4: M_pp not positive definite; bit 8: K_p^T M_pp^-1 K_p singular
    if (tid == 0 && bad) atomicOr(it.flag, ((bad & 1) ? 4 : 0) | ((bad & 2) ? 8 : 0));
}

// ---------------------------------------------------------------------------
// small-body preconditioner: apply (grid.y = right-hand side)
// ---------------------------------------------------------------------------

// Solves one body's [M_pp -K_p; -K_p^T 0][lambda; U] = [s; bottom] with the
// body's factor staged in LDS (lds: m(m+1)/2 + 6m + 36 doubles of the
// factor, then 2m doubles).  With a rotation R (shared reference-shape factor), the
// inputs are taken into the body frame (R^T on every 3-vector: blob
// velocities, force, torque) and the results back (R on lambda, u, omega):
// the RPY tensor and K are rotation-covariant, M_pp = R~ M_ref R~^T and
// K_p = R~ K_ref diag(R, R)^T.
constexpr int kApplyThreads = 256;  // four waves: more factor loads in flight per body
constexpr int kRowLanes = 4;        // lanes per row in the triangular products

// Sum over the kRowLanes adjacent lanes of a row (all lanes take part).
__device__ __forceinline__ double sum_row_lanes(double v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    return v;
}

// With `resist` (resistance problem) only lambda = M_pp^-1 s is formed:
// bot_in and U_out are not touched.
__device__ __forceinline__ void precond_body_apply(const BodyWork &it, const gmem<const double> s_in,
                                                   const gmem<const double> bot_in, const gmem<double> lam_out,
                                                   const gmem<double> U_out, double *lds, double *g, bool resist) {
    const int m = 3 * it.n_blobs, tid = threadIdx.x;
    // the whole factor [Li | Y | S^-1] is staged in LDS, eight loads in
    // flight per thread, followed by the right-hand side
    const int np = m * (m + 1) / 2, nf = np + 6 * m + 36;
    double *F = lds, *sv = lds + nf, *t = sv + m;
    const double *Li = F, *Y = F + np, *Si = F + np + 6 * m;  // Li packed by columns
    for (int e0 = tid; e0 < nf; e0 += 8 * kApplyThreads) {
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = e0 + i * kApplyThreads;
            v[i] = e < nf ? as_global(it.factor)[e] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = e0 + i * kApplyThreads;
            if (e < nf) F[e] = v[i];
        }
    }
    const gmem<const double> R = as_global(it.rot);
    if (it.rot) {
        for (int e = tid; e < m; e += kApplyThreads) {
            const int b = e - e % 3, c = e % 3;
            sv[e] = R[c] * s_in[b] + R[3 + c] * s_in[b + 1] + R[6 + c] * s_in[b + 2];
        }
    } else {
        for (int e = tid; e < m; e += kApplyThreads) sv[e] = s_in[e];
    }
    __syncthreads();
    // The triangular products give each row's sum to kRowLanes adjacent
    // lanes (every lane runs the same iterations, so the shuffles that
    // combine a row's parts see all of its lanes).
    const int part = tid % kRowLanes;
    // t = Li s
    for (int base = 0; base < m; base += kApplyThreads / kRowLanes) {
        const int r = base + tid / kRowLanes;
        double acc = 0.0;
        if (r < m)
            for (int c = part; c <= r; c += kRowLanes) acc += Li[packed_col(m, c) + r - c] * sv[c];
        acc = sum_row_lanes(acc);
        if (r < m && part == 0) t[r] = acc;
    }
    __syncthreads();
    // g = F - Y^T t, F = -bottom: 32 lanes per component
    if (!resist) {
        const int k = tid / 32, p32 = tid % 32;
        double acc = 0.0;
        if (k < 6)
            for (int l = p32; l < m; l += 32) acc += Y[l * 6 + k] * t[l];
        for (int off = 16; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (k < 6 && p32 == 0) {
            double bot = bot_in[k];
            if (it.rot) {
                const int b = k - k % 3, c = k % 3;
                bot = R[c] * bot_in[b] + R[3 + c] * bot_in[b + 1] + R[6 + c] * bot_in[b + 2];
            }
            g[k] = -bot - acc;
        }
    }
    __syncthreads();
    // U = S^-1 g (U = 0 for the resistance problem)
    if (tid < 6) {
        double u = 0.0;
        if (!resist)
            for (int k = 0; k < 6; ++k) u += Si[tid * 6 + k] * g[k];
        g[6 + tid] = u;
    }
    __syncthreads();
    // w = t + Y U (into sv), then lambda = Li^T w
    for (int r = tid; r < m; r += kApplyThreads) {
        double acc = t[r];
        for (int k = 0; k < 6; ++k) acc += Y[r * 6 + k] * g[6 + k];
        sv[r] = acc;
    }
    __syncthreads();
    // lambda = Li^T w (into t when it still has to be rotated)
    for (int base = 0; base < m; base += kApplyThreads / kRowLanes) {
        const int r = base + tid / kRowLanes;
        double acc = 0.0;
        if (r < m)
            for (int c = r + part; c < m; c += kRowLanes) acc += Li[packed_col(m, r) + c - r] * sv[c];
        acc = sum_row_lanes(acc);
        if (r < m && part == 0) {
            if (it.rot) t[r] = acc;
            else lam_out[r] = acc;
        }
    }
    if (!it.rot) {
        if (tid < 6 && !resist) U_out[tid] = g[6 + tid];
        return;
    }
    __syncthreads();
    for (int e = tid; e < m; e += kApplyThreads) {
        const int b = e - e % 3, c = e % 3;
        lam_out[e] = R[3 * c] * t[b] + R[3 * c + 1] * t[b + 1] + R[3 * c + 2] * t[b + 2];
    }
    if (tid < 6 && !resist) {
        const int b = 6 + tid - tid % 3, c = tid % 3;
        U_out[tid] = R[3 * c] * g[b] + R[3 * c + 1] * g[b + 1] + R[3 * c + 2] * g[b + 2];
    }
}

__global__ __launch_bounds__(kApplyThreads) void precond_apply_small_kernel(const PrecondApplyJob *__restrict__ jobs,
                                                                 int32_t n_jobs) {
    extern __shared__ double lds[];
    __shared__ double g[12];
    const int64_t w = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= w) lo = mid; else hi = mid - 1;
    }
    const PrecondApplyJob &J = jobs[lo];
    const int64_t rhs = blockIdx.y;
    if (rhs >= J.nrhs) return;
    const BodyWork it = J.items[w - J.wg_begin];
    const gmem<const double> in = as_global(J.in + rhs * J.ld);
    gmem<double> out = as_global(J.out + rhs * J.ld);
    const int64_t b3 = 3 * it.blob0;
    const int64_t u6 = J.mode ? 0 : J.nb3 + 6 * (int64_t)it.body;
    precond_body_apply(it, in + b3, in + u6, out + b3, out + u6, lds, g, J.mode != 0);
}

// ---------------------------------------------------------------------------
// resistance problem: right-hand side K U + slip, and F = K^T lambda
// ---------------------------------------------------------------------------

__global__ void build_rhs_resist_kernel(const double *__restrict__ U, const double *__restrict__ slip,
                                        const double *__restrict__ pos, const double *__restrict__ q,
                                        const int32_t *__restrict__ blob_body, int64_t nb, double *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int64_t p = as_global(blob_body)[i];
    const gmem<const double> u = as_global(U) + 6 * p, qp = as_global(q) + 3 * p, r = as_global(pos) + 3 * i;
    const double d[3] = {r[0] - qp[0], r[1] - qp[1], r[2] - qp[2]};
    double v[3] = {u[0] + u[4] * d[2] - u[5] * d[1], u[1] + u[5] * d[0] - u[3] * d[2],
                   u[2] + u[3] * d[1] - u[4] * d[0]};
    if (slip)
        for (int c = 0; c < 3; ++c) v[c] += as_global(slip)[3 * i + c];
    for (int c = 0; c < 3; ++c) as_global(b)[3 * i + c] = v[c];
}

hipError_t launch_build_rhs_resist(const double *U, const double *slip, const double *pos, const double *q,
                                   const int32_t *blob_body, int64_t nb, double *b, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(build_rhs_resist_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, U, slip, pos, q,
                       blob_body, nb, b);
    return hipGetLastError();
}

// One wave per body: force sum and torque about q_p, reduced across lanes
// in a fixed order.
__global__ void body_forces_kernel(const double *__restrict__ pos, const double *__restrict__ q,
                                   const int64_t *__restrict__ body_off, const double *__restrict__ lam,
                                   double *__restrict__ F) {
    const int64_t p = blockIdx.x;
    const int64_t b0 = as_global(body_off)[p], b1 = as_global(body_off)[p + 1];
    const gmem<const double> qp = as_global(q) + 3 * p;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 64) {
        const gmem<const double> l = as_global(lam) + 3 * i, r = as_global(pos) + 3 * i;
        const double d[3] = {r[0] - qp[0], r[1] - qp[1], r[2] - qp[2]};
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
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) as_global(F)[6 * p + k] = acc[k];
}

hipError_t launch_body_forces(const double *pos, const double *q, const int64_t *body_off, const double *lam,
                              int64_t N, double *F, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(body_forces_kernel, dim3((unsigned)N), dim3(64), 0, s, pos, q, body_off, lam, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// body orientations
// ---------------------------------------------------------------------------

// R of the unit quaternion q / |q| (w, x, y, z), row-major; the factor
// s = 2 / |q|^2 folds the normalisation into the usual formula.
__global__ void quat_rot_kernel(const double *__restrict__ quat, int64_t N, double *__restrict__ rot, int *flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const gmem<const double> Q = as_global(quat) + 4 * p;
    const double w = Q[0], x = Q[1], y = Q[2], z = Q[3];
    const double n2 = w * w + x * x + y * y + z * z;
    gmem<double> R = as_global(rot) + 9 * p;
    if (!(n2 > 0.0) || !isfinite(n2)) {
        atomicOr(flag, 16);
        for (int e = 0; e < 9; ++e) R[e] = (e % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    const double s = 2.0 / n2;
    R[0] = 1.0 - s * (y * y + z * z);
    R[1] = s * (x * y - w * z);
    R[2] = s * (x * z + w * y);
    R[3] = s * (x * y + w * z);
    R[4] = 1.0 - s * (x * x + z * z);
    R[5] = s * (y * z - w * x);
    R[6] = s * (x * z - w * y);
    R[7] = s * (y * z + w * x);
    R[8] = 1.0 - s * (x * x + y * y);
}

hipError_t launch_quat_rotations(const double *quat, int64_t N, double *rot, int *flag, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(quat_rot_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, quat, N, rot, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// saddle-point operator around the pair product
// ---------------------------------------------------------------------------

// Blob rows: y_lambda[i] = pref * sum_s partial[s][i] - (u_p + omega_p x (r_i - q_p)),
// or with `resid`, r_lambda[i] = b_lambda[i] - y_lambda[i].
__global__ void saddle_blob_kernel(const SaddleJob *__restrict__ jobs, int32_t n_jobs) {
    // one workgroup covers 256 blobs of one job; job located by prefix
    const int64_t w = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].blk_begin <= w) lo = mid; else hi = mid - 1;
    }
    const SaddleJob &J = jobs[lo];
    const int64_t i = (w - J.blk_begin) * 256 + threadIdx.x;
    if (i >= J.nb) return;
    double v[3] = {0.0, 0.0, 0.0};
    const int64_t n3 = 3 * J.nb;
    for (int32_t s = 0; s < J.n_split; ++s) {
        const gmem<const double> p = as_global(J.partial + s * n3 + 3 * i);
        v[0] += p[0];
        v[1] += p[1];
        v[2] += p[2];
    }
    v[0] *= J.pref, v[1] *= J.pref, v[2] *= J.pref;
    saddle_blob_row(J, i, v);
}

// Body rows: y_U[p] = -(sum_i lambda_i, sum_i (r_i - q_p) x lambda_i), or the
// residual b_U - y_U.  One wave per body.
__global__ void saddle_body_kernel(const SaddleJob *__restrict__ jobs, int32_t n_jobs) {
    saddle_body_rows(jobs, n_jobs, blockIdx.x, threadIdx.x);
}

hipError_t launch_precond_build_small(const BodyWork *items, int32_t n_items, int max_m, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    // m^2 + 13m + 36 doubles: 65,472 bytes at the largest small body (m = 84)
    size_t lds = ((size_t)max_m * max_m + 13 * (size_t)max_m + 36) * sizeof(double);
    hipLaunchKernelGGL(precond_build_small_kernel, dim3(n_items), dim3(64), lds, s, items, n_items);
    return hipGetLastError();
}

hipError_t launch_precond_apply_small(const PrecondApplyJob *jobs, int32_t n_jobs, int64_t n_wg,
                                      int32_t max_rhs, int max_m, hipStream_t s) {
    if (n_wg <= 0 || max_rhs <= 0) return hipSuccess;
    size_t lds = ((size_t)max_m * (max_m + 1) / 2 + 8 * max_m + 36) * sizeof(double);  // packed L^-1, Y, S^-1, 2m
    hipLaunchKernelGGL(precond_apply_small_kernel, dim3((unsigned)n_wg, max_rhs), dim3(kApplyThreads), lds, s, jobs,
                       n_jobs);
    return hipGetLastError();
}

hipError_t launch_saddle(const SaddleJob *jobs, int32_t n_jobs, int64_t n_blob_blocks, int64_t n_bodies,
                         hipStream_t s) {
    if (n_blob_blocks > 0)
        hipLaunchKernelGGL(saddle_blob_kernel, dim3((unsigned)n_blob_blocks), dim3(256), 0, s, jobs, n_jobs);
    if (n_bodies > 0)
        hipLaunchKernelGGL(saddle_body_kernel, dim3((unsigned)n_bodies), dim3(64), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

}  // namespace rmb

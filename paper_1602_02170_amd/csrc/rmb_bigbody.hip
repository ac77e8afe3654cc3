// Preconditioner build and apply for bodies whose 3n x 3n mobility block is
// too large for LDS (Sec. 2.2.2: the per-body factorisation of M_pp behind
// eq:saddle_M_precon), e.g. 162-blob shells (486 x 486).
//
// Storage per body, leading dimension Mp = m rounded up to the panel width
// NB (padding rows/columns hold the identity, so the padded factor is
// blockdiag(L, I)):
//   L  : Mp x Mp, column-major, lower triangle
//   Y  : Mp x 6, row-major  (L^-1 K_p, zero in the padding)
//   Sc : 6 x 6 lower        (Cholesky factor of Y^T Y)
//
// Factorisation: one workgroup (4 waves) per body, all bodies in one launch,
// left-looking by panels of NB columns.  Panel update
//   A[j:, j:j+NB] -= L[j:, 0:j] L[j:j+NB, 0:j]^T
// runs on FP64 matrix cores (v_mfma_f64_16x16x4: D[16x16] += A[16x4] B[4x16])
// with operands read straight from global memory, so each column block of L
// is read once per later panel and the trailing matrix is never rewritten.
// The panel's NB x NB diagonal block is then factorised in LDS and the rows
// below it are solved against it (one row per lane, registers).
#include <cmath>

#include "rmb_blocks.h"
#include "rmb_body.h"

namespace rmb {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Lane layout of v_mfma_f64_16x16x4f64 (one wave):
//   A operand: lane holds A[lane % 16][lane / 16]
//   B operand: lane holds B[lane / 16][lane % 16]
//   C/D:       lane holds D[lane / 16 + 4 r][lane % 16], r = 0..3 (measured on gfx950)
__device__ __forceinline__ dbl4 mfma16x16x4(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}


// ---------------------------------------------------------------------------
// assembly of the padded block (column-major), grid = (body, chunk)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void assemble_large_kernel(const BigBody *__restrict__ items) {
    const BigBody it = items[blockIdx.x];
    const int n = it.w.n_blobs, m = 3 * n, Mp = it.Mp;
    double *A = it.w.factor;
    const int64_t npairs = (int64_t)n * n;
    for (int64_t pq = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; pq < npairs;
         pq += (int64_t)gridDim.y * blockDim.x) {
        const int i = (int)(pq / n), j = (int)(pq % n);
        const double *ri = it.w.pos + 3 * (it.w.blob0 + i);
        const double *rj = it.w.pos + 3 * (it.w.blob0 + j);
        const double a_i[3] = {ri[0], ri[1], ri[2]}, a_j[3] = {rj[0], rj[1], rj[2]};
        double B[9];
        pair_block_f64(a_i, a_j, it.w.a, it.w.wall != 0, B);
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) A[(int64_t)(3 * j + q) * Mp + 3 * i + p] = it.w.pref * B[3 * p + q];
    }
    // identity padding
    const int64_t pad = (int64_t)Mp * Mp - (int64_t)m * Mp;  // columns m..Mp-1 entirely
    for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < pad; e += (int64_t)gridDim.y * blockDim.x) {
        const int64_t col = m + e / Mp, row = e % Mp;
        A[col * Mp + row] = row == col ? 1.0 : 0.0;
    }
    // rows m..Mp-1 of columns 0..m-1
    const int64_t padr = (int64_t)(Mp - m) * m;
    for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < padr; e += (int64_t)gridDim.y * blockDim.x) {
        const int64_t col = e / (Mp - m), row = m + e % (Mp - m);
        A[col * Mp + row] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// left-looking blocked Cholesky with MFMA panel updates
// ---------------------------------------------------------------------------

template <int NB>
__global__ __launch_bounds__(256) void chol_large_kernel(const BigBody *__restrict__ items) {
    constexpr int CT = NB / 16;  // column tiles per panel
    constexpr int G = 4;         // row tiles per wave per pass
    __shared__ double D[NB * NB];
    __shared__ int bad;
    const BigBody it = items[blockIdx.x];
    const int Mp = it.Mp;
    double *L = it.w.factor;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    if (tid == 0) bad = 0;

    for (int j = 0; j < Mp; j += NB) {
        // 1. panel update: rows [j, Mp), columns [j, j+NB)
        const int RT = (Mp - j) / 16;  // row tiles in the panel
        for (int pass = 0; pass * 4 * G < RT; ++pass) {
            dbl4 acc[G][CT];
            int row0[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int t = pass * 4 * G + g * 4 + wave;
                row0[g] = t < RT ? j + 16 * t : -1;
#pragma unroll
                for (int c = 0; c < CT; ++c) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc[g][c][r] = row0[g] >= 0 ? L[(int64_t)(j + 16 * c + l16) * Mp + row0[g] + l4 + 4 * r] : 0.0;
                }
            }
            for (int k0 = 0; k0 < j; k0 += 4) {
                const int64_t kcol = (int64_t)(k0 + l4) * Mp;
                double b[CT];
#pragma unroll
                for (int c = 0; c < CT; ++c) b[c] = L[kcol + j + 16 * c + l16];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    if (row0[g] < 0) continue;
                    const double a = -L[kcol + row0[g] + l16];
#pragma unroll
                    for (int c = 0; c < CT; ++c) acc[g][c] = mfma16x16x4(a, b[c], acc[g][c]);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (row0[g] < 0) continue;
#pragma unroll
                for (int c = 0; c < CT; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        L[(int64_t)(j + 16 * c + l16) * Mp + row0[g] + l4 + 4 * r] = acc[g][c][r];
            }
        }
        __syncthreads();
        // 2. factorise the diagonal block in LDS
        for (int e = tid; e < NB * NB; e += 256) {
            const int r = e % NB, c = e / NB;
            D[c * NB + r] = L[(int64_t)(j + c) * Mp + j + r];
        }
        __syncthreads();
        for (int c = 0; c < NB; ++c) {
            if (tid == 0) {
                const double d = D[c * NB + c];
                if (!(d > 0.0)) bad = 1;
                D[c * NB + c] = sqrt(d > 0.0 ? d : 1.0);
            }
            __syncthreads();
            const double dc = D[c * NB + c];
            for (int r = c + 1 + tid; r < NB; r += 256) D[c * NB + r] /= dc;
            __syncthreads();
            const int rem = NB - c - 1;
            for (int e = tid; e < rem * rem; e += 256) {
                const int r = c + 1 + e % rem, cc = c + 1 + e / rem;
                if (r >= cc) D[cc * NB + r] -= D[c * NB + r] * D[c * NB + cc];
            }
            __syncthreads();
        }
        for (int e = tid; e < NB * NB; e += 256) {
            const int r = e % NB, c = e / NB;
            L[(int64_t)(j + c) * Mp + j + r] = r >= c ? D[c * NB + r] : 0.0;
        }
        // 3. rows below: x L11^T = a  (one row per lane)
        for (int r = j + NB + tid; r < Mp; r += 256) {
            double x[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) x[c] = L[(int64_t)(j + c) * Mp + r];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                double v = x[c];
#pragma unroll
                for (int l = 0; l < c; ++l) v -= x[l] * D[l * NB + c];
                x[c] = v / D[c * NB + c];
            }
#pragma unroll
            for (int c = 0; c < NB; ++c) L[(int64_t)(j + c) * Mp + r] = x[c];
        }
        // zero the strict upper triangle of the panel's columns above the diagonal block
        for (int e = tid; e < j * NB; e += 256) {
            const int r = e % j, c = e / j;
            L[(int64_t)(j + c) * Mp + r] = 0.0;
        }
        __syncthreads();
    }
    if (tid == 0 && bad) atomicOr(it.w.flag, 4);
}

// ---------------------------------------------------------------------------
// blocked triangular solves with R right-hand sides held in LDS (row-major
// Mp x R), panels of NB
// ---------------------------------------------------------------------------

// X <- L^-1 X
template <int NB, int R>
__device__ void forward_blocked(const double *__restrict__ L, int Mp, double *X, double *D) {
    const int tid = threadIdx.x;
    for (int j = 0; j < Mp; j += NB) {
        // X[j:j+NB] -= L[j:j+NB, 0:j] X[0:j]
        for (int o = tid; o < NB * R; o += 256) {
            const int r = o / R, c = o % R;
            double acc = 0.0;
            for (int k = 0; k < j; ++k) acc += L[(int64_t)k * Mp + j + r] * X[k * R + c];
            X[(j + r) * R + c] -= acc;
        }
        for (int e = tid; e < NB * NB; e += 256) {
            const int r = e % NB, c = e / NB;
            D[c * NB + r] = L[(int64_t)(j + c) * Mp + j + r];
        }
        __syncthreads();
        // forward substitution with the diagonal block, one thread per rhs
        if (tid < R) {
            for (int r = 0; r < NB; ++r) {
                double v = X[(j + r) * R + tid];
                for (int l = 0; l < r; ++l) v -= D[l * NB + r] * X[(j + l) * R + tid];
                X[(j + r) * R + tid] = v / D[r * NB + r];
            }
        }
        __syncthreads();
    }
}

// X <- L^-T X
template <int NB, int R>
__device__ void backward_blocked(const double *__restrict__ L, int Mp, double *X, double *D) {
    const int tid = threadIdx.x;
    for (int j = Mp - NB; j >= 0; j -= NB) {
        // X[j:j+NB] -= L[j+NB:Mp, j:j+NB]^T X[j+NB:Mp]
        for (int o = tid; o < NB * R; o += 256) {
            const int cc = o / R, c = o % R;
            double acc = 0.0;
            const double *col = L + (int64_t)(j + cc) * Mp;
            for (int k = j + NB; k < Mp; ++k) acc += col[k] * X[k * R + c];
            X[(j + cc) * R + c] -= acc;
        }
        for (int e = tid; e < NB * NB; e += 256) {
            const int r = e % NB, c = e / NB;
            D[c * NB + r] = L[(int64_t)(j + c) * Mp + j + r];
        }
        __syncthreads();
        if (tid < R) {
            for (int r = NB - 1; r >= 0; --r) {
                double v = X[(j + r) * R + tid];
                for (int l = r + 1; l < NB; ++l) v -= D[r * NB + l] * X[(j + l) * R + tid];
                X[(j + r) * R + tid] = v / D[r * NB + r];
            }
        }
        __syncthreads();
    }
}

// Y = L^-1 K_p, S = Y^T Y, Sc = chol(S); one workgroup per body.
template <int NB>
__global__ __launch_bounds__(256) void project_large_kernel(const BigBody *__restrict__ items) {
    extern __shared__ double lds[];
    __shared__ double D[NB * NB];
    __shared__ double S[36];
    __shared__ int bad;
    const BigBody it = items[blockIdx.x];
    const int Mp = it.Mp, m = 3 * it.w.n_blobs, tid = threadIdx.x;
    const double *L = it.w.factor;
    double *Y = lds;  // Mp x 6
    if (tid == 0) bad = 0;
    const double *q = it.w.q;
    for (int e = tid; e < 6 * Mp; e += 256) {
        const int row = e / 6, k = e % 6;
        double v = 0.0;
        if (row < m) {
            const int i = row / 3, c = row % 3;
            const double *ri = it.w.pos + 3 * (it.w.blob0 + i);
            const double d[3] = {ri[0] - q[0], ri[1] - q[1], ri[2] - q[2]};
            v = K_entry(d, c, k);
        }
        Y[e] = v;
    }
    __syncthreads();
    forward_blocked<NB, 6>(L, Mp, Y, D);
    if (tid < 36) {
        const int r = tid / 6, c = tid % 6;
        double acc = 0.0;
        for (int l = 0; l < Mp; ++l) acc += Y[l * 6 + r] * Y[l * 6 + c];
        S[tid] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        for (int j = 0; j < 6; ++j) {
            double dj = S[j * 6 + j];
            for (int k = 0; k < j; ++k) dj -= S[j * 6 + k] * S[j * 6 + k];
            if (!(dj > 0.0)) {
                bad = 1;
                dj = 1.0;
            }
            const double ljj = sqrt(dj);
            S[j * 6 + j] = ljj;
            for (int i = j + 1; i < 6; ++i) {
                double v = S[i * 6 + j];
                for (int k = 0; k < j; ++k) v -= S[i * 6 + k] * S[j * 6 + k];
                S[i * 6 + j] = v / ljj;
            }
        }
    }
    __syncthreads();
    double *Yg = it.w.factor + (int64_t)Mp * Mp;
    for (int e = tid; e < 6 * Mp; e += 256) Yg[e] = Y[e];
    double *Sc = Yg + 6 * Mp;
    if (tid < 36) Sc[tid] = ((tid % 6) <= (tid / 6)) ? S[tid] : 0.0;
    if (tid == 0 && bad) atomicOr(it.w.flag, 8);
}

// Apply P^-1 to up to 8 right-hand sides of one body per workgroup
// (grid.y = groups of 8 rhs).  lds: X (Mp x 8).
template <int NB>
__global__ __launch_bounds__(256) void apply_large_kernel(const PrecondApplyJob *__restrict__ jobs, int32_t n_jobs) {
    extern __shared__ double lds[];
    __shared__ double D[NB * NB];
    __shared__ double g[8][6];
    const int64_t w = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= w) lo = mid; else hi = mid - 1;
    }
    const PrecondApplyJob &J = jobs[lo];
    const BigBody it = ((const BigBody *)J.items)[w - J.wg_begin];
    const int Mp = it.Mp, m = 3 * it.w.n_blobs, tid = threadIdx.x;
    const int r0 = 8 * blockIdx.y;
    const int R = min(8, J.nrhs - r0);
    if (R <= 0) return;
    const double *L = it.w.factor;
    const double *Y = L + (int64_t)Mp * Mp, *Sc = Y + 6 * Mp;
    double *X = lds;  // Mp x 8
    const int64_t b3 = 3 * it.w.blob0, u6 = J.nb3 + 6 * (int64_t)it.w.body;
    for (int e = tid; e < Mp * 8; e += 256) {
        const int row = e / 8, c = e % 8;
        X[e] = (row < m && c < R) ? J.in[(int64_t)(r0 + c) * J.ld + b3 + row] : 0.0;
    }
    __syncthreads();
    forward_blocked<NB, 8>(L, Mp, X, D);
    // g = F - Y^T t, F = -bottom
    if (tid < 48) {
        const int c = tid / 6, k = tid % 6;
        if (c < R) {
            double acc = 0.0;
            for (int l = 0; l < Mp; ++l) acc += Y[l * 6 + k] * X[l * 8 + c];
            g[c][k] = -J.in[(int64_t)(r0 + c) * J.ld + u6 + k] - acc;
        }
    }
    __syncthreads();
    if (tid < R) {
        double u[6];
        double *gg = g[tid];
        for (int i = 0; i < 6; ++i) {
            double v = gg[i];
            for (int k = 0; k < i; ++k) v -= Sc[i * 6 + k] * u[k];
            u[i] = v / Sc[i * 6 + i];
        }
        for (int i = 5; i >= 0; --i) {
            double v = u[i];
            for (int k = i + 1; k < 6; ++k) v -= Sc[k * 6 + i] * gg[k];
            gg[i] = v / Sc[i * 6 + i];
        }
    }
    __syncthreads();
    for (int e = tid; e < Mp * 8; e += 256) {
        const int row = e / 8, c = e % 8;
        if (c < R) {
            double acc = X[e];
            for (int k = 0; k < 6; ++k) acc += Y[row * 6 + k] * g[c][k];
            X[e] = acc;
        }
    }
    __syncthreads();
    backward_blocked<NB, 8>(L, Mp, X, D);
    for (int e = tid; e < m * 8; e += 256) {
        const int row = e / 8, c = e % 8;
        if (c < R) J.out[(int64_t)(r0 + c) * J.ld + b3 + row] = X[e];
    }
    if (tid < 48) {
        const int c = tid / 6, k = tid % 6;
        if (c < R) J.out[(int64_t)(r0 + c) * J.ld + u6 + k] = g[c][k];
    }
}

// ---------------------------------------------------------------------------

int large_panel_width(int variant) { return variant == 1 ? 32 : 16; }

hipError_t launch_precond_build_large(const BigBody *items, int32_t n_items, int max_Mp, int variant, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(assemble_large_kernel, dim3(n_items, 16), dim3(256), 0, s, items);
    const size_t lds = (size_t)max_Mp * 6 * sizeof(double);
    if (variant == 1) {
        hipLaunchKernelGGL(chol_large_kernel<32>, dim3(n_items), dim3(256), 0, s, items);
        hipLaunchKernelGGL(project_large_kernel<32>, dim3(n_items), dim3(256), lds, s, items);
    } else {
        hipLaunchKernelGGL(chol_large_kernel<16>, dim3(n_items), dim3(256), 0, s, items);
        hipLaunchKernelGGL(project_large_kernel<16>, dim3(n_items), dim3(256), lds, s, items);
    }
    return hipGetLastError();
}

hipError_t launch_precond_apply_large(const PrecondApplyJob *jobs, int32_t n_jobs, int64_t n_wg, int32_t max_rhs,
                                      int max_Mp, int variant, hipStream_t s) {
    if (n_wg <= 0 || max_rhs <= 0) return hipSuccess;
    const size_t lds = (size_t)max_Mp * 8 * sizeof(double);
    dim3 g((unsigned)n_wg, (max_rhs + 7) / 8);
    if (variant == 1)
        hipLaunchKernelGGL(apply_large_kernel<32>, g, dim3(256), lds, s, jobs, n_jobs);
    else
        hipLaunchKernelGGL(apply_large_kernel<16>, g, dim3(256), lds, s, jobs, n_jobs);
    return hipGetLastError();
}

}  // namespace rmb

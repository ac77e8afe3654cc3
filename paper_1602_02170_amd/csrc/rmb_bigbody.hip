// Preconditioner build and apply for bodies whose 3n x 3n mobility block is
// too large for LDS (Sec. 2.2.2: the per-body factorisation of M_pp behind
// eq:saddle_M_precon), e.g. 162-blob shells (486 x 486).
//
// Storage per body (doubles), Mp = 3n rounded up to 32; rows and columns
// past 3n hold the identity, so the padded factor is blockdiag(L, I):
//   L    : Mp x Mp, column-major, lower triangle (the upper triangle is zero)
//   Y    : Mp x 6, row-major (L^-1 K_p, zero in the padding)
//   Dinv : the inverses of L's NB x NB diagonal blocks, block j/NB at
//          offset j*NB, each column-major (room for NB = 32: Mp x 32)
//   Sc   : 6 x 6 lower (Cholesky factor of S = Y^T Y)
//
// Build, each launch covering all bodies: assembly of the lower triangle,
// Cholesky (with the diagonal-block inverses), projection (Y, S, Sc).
//
// Cholesky: one workgroup (4 waves) per body, left-looking by panels of NB
// columns.  Panel update
//   A[j:, j:j+NB] -= L[j:, 0:j] L[j:j+NB, 0:j]^T
// runs on FP64 matrix cores (v_mfma_f64_16x16x4: D[16x16] += A[16x4] B[4x16]);
// the operands of the next 16 columns of L are loaded while the current ones
// are multiplied.  The panel's NB x NB diagonal block is then factorised in
// LDS (one barrier per column) and inverted, and the rows below it become
// x = a L11^-T, a product with the inverse, also on matrix cores.
//
// Substitutions (projection and apply) go by panels, right-looking: the
// panel's unknowns are x_j = Dinv_j b_j, then every later (earlier, for
// L^T) row is updated at once, with all of its loads in flight.
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

constexpr int kDinvCols = 32;  // room reserved per row for the diagonal-block inverses

__device__ __forceinline__ double *big_Y(const BigBody &it) { return it.w.factor + (int64_t)it.Mp * it.Mp; }
__device__ __forceinline__ double *big_Dinv(const BigBody &it) { return big_Y(it) + 6 * (int64_t)it.Mp; }
__device__ __forceinline__ double *big_Sc(const BigBody &it) { return big_Dinv(it) + (int64_t)kDinvCols * it.Mp; }

// ---------------------------------------------------------------------------
// assembly of the lower triangle of the padded block (column-major)
// ---------------------------------------------------------------------------

constexpr int kAsmBlobs = 16;      // blobs per tile side (48 x 48 entries)
constexpr int kAsmPadGroups = 8;   // workgroups per body writing the padding

int asm_tiles(int max_Mp) {
    const int T = (max_Mp / 3 + kAsmBlobs - 1) / kAsmBlobs;
    return T * (T + 1) / 2 + kAsmPadGroups;
}

// grid = (body, tile): tile y < T(T+1)/2 is the blob-block pair (I, J),
// I >= J, y = I(I+1)/2 + J; each thread forms one 3x3 pair block into an
// LDS tile, which is then written out column by column.  The next
// kAsmPadGroups tiles write the identity padding.
__global__ __launch_bounds__(256) void assemble_large_kernel(const BigBody *__restrict__ items) {
    constexpr int E = 3 * kAsmBlobs;
    __shared__ double tile[E][E + 1];  // [column][row]
    const BigBody it = items[blockIdx.x];
    const int n = it.w.n_blobs, m = 3 * n, Mp = it.Mp;
    gmem<double> A = as_global(it.w.factor);
    const int T = (n + kAsmBlobs - 1) / kAsmBlobs;
    const int ntile = T * (T + 1) / 2;
    const int y = blockIdx.y, tid = threadIdx.x;
    if (y < ntile) {
        int I = (int)((sqrt(8.0 * y + 1.0) - 1.0) * 0.5);
        while ((I + 1) * (I + 2) / 2 <= y) ++I;
        while (I * (I + 1) / 2 > y) --I;
        const int J = y - I * (I + 1) / 2;
        const int il = tid % kAsmBlobs, jl = tid / kAsmBlobs;
        const int i = I * kAsmBlobs + il, j = J * kAsmBlobs + jl;
        if (i < n && j < n) {
            const gmem<const double> ri = as_global(it.w.pos + 3 * (it.w.blob0 + i));
            const gmem<const double> rj = as_global(it.w.pos + 3 * (it.w.blob0 + j));
            const double a_i[3] = {ri[0], ri[1], ri[2]}, a_j[3] = {rj[0], rj[1], rj[2]};
            double B[9];
            pair_block_f64(a_i, a_j, it.w.a, it.w.wall != 0, B);
            // permeable bodies: d_i on the diagonal (eq:permeable_slip)
            const double d = (i == j && it.w.shift) ? as_global(it.w.shift)[it.w.blob0 + i] : 0.0;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q)
                    tile[3 * jl + q][3 * il + p] = it.w.pref * B[3 * p + q] + (p == q ? d : 0.0);
        }
        __syncthreads();
        const int r0 = E * I, c0 = E * J;
        for (int e = tid; e < E * E; e += 256) {
            const int c = e / E, r = e % E;
            if (r0 + r < m && c0 + c < m) A[(int64_t)(c0 + c) * Mp + r0 + r] = tile[c][r];
        }
        return;
    }
    const int g = y - ntile;
    if (g >= kAsmPadGroups) return;
    const int64_t stride = (int64_t)kAsmPadGroups * 256;
    // columns m..Mp-1: identity
    const int64_t pad = (int64_t)(Mp - m) * Mp;
    for (int64_t e = (int64_t)g * 256 + tid; e < pad; e += stride) {
        const int64_t col = m + e / Mp, row = e % Mp;
        A[col * Mp + row] = row == col ? 1.0 : 0.0;
    }
    // rows m..Mp-1 of columns 0..m-1: zero
    const int64_t padr = (int64_t)(Mp - m) * m;
    for (int64_t e = (int64_t)g * 256 + tid; e < padr; e += stride) {
        const int64_t col = e / (Mp - m), row = m + e % (Mp - m);
        A[col * Mp + row] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// left-looking blocked Cholesky with MFMA panel updates
// ---------------------------------------------------------------------------

// NB: panel width; G: 16-row tiles per wave per pass; U: steps of 4 columns
// per prefetched chunk (the autotuner picks among a few shapes).
template <int NB, int G, int U>
__global__ __launch_bounds__(256) void chol_large_kernel(const BigBody *__restrict__ items) {
    constexpr int CT = NB / 16;  // column tiles per panel
    __shared__ double D[NB * NB];   // diagonal block being factorised (column-major)
    __shared__ double Lc[NB * NB];  // its Cholesky factor
    __shared__ double W[NB * NB];   // the factor's inverse
    __shared__ double Li[NB];       // reciprocals of the factor's diagonal
    __shared__ int bad;
    const BigBody it = items[blockIdx.x];
    const int Mp = it.Mp;
    const gmem<double> L = as_global(it.w.factor);
    const gmem<double> Dinv = as_global(big_Dinv(it));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    if (tid == 0) bad = 0;

    for (int j = 0; j < Mp; j += NB) {
        // 1. panel update: rows [j, Mp), columns [j, j+NB).  A wave's row
        //    tiles past the panel are clamped to its last tile, so every load
        //    is unconditional (no branch between a prefetch and its use);
        //    only their stores are skipped.
        const int RT = (Mp - j) / 16;  // row tiles in the panel
        for (int pass = 0; pass * 4 * G < RT; ++pass) {
            dbl4 acc[G][CT];
            int row0[G];
            bool live[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int t = pass * 4 * G + g * 4 + wave;
                live[g] = t < RT;
                row0[g] = j + 16 * (t < RT ? t : RT - 1);
#pragma unroll
                for (int c = 0; c < CT; ++c) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc[g][c][r] = L[(j + 16 * c + l16) * Mp + row0[g] + l4 + 4 * r];
                }
            }
            if (j > 0) {
                // j is a multiple of 16 (and of 4 * U): nch whole chunks
                const int nch = j / (4 * U);
                double a0[U][G], b0[U][CT], a1[U][G], b1[U][CT];
                auto load = [&](int ch, double (&a)[U][G], double (&b)[U][CT]) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int kc = (4 * U * ch + 4 * u + l4) * Mp;  // Mp^2 < 2^31
#pragma unroll
                        for (int c = 0; c < CT; ++c) b[u][c] = L[kc + j + 16 * c + l16];
#pragma unroll
                        for (int g = 0; g < G; ++g) a[u][g] = -L[kc + row0[g] + l16];
                    }
                };
                auto mma = [&](const double (&a)[U][G], const double (&b)[U][CT]) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int g = 0; g < G; ++g)
#pragma unroll
                            for (int c = 0; c < CT; ++c) acc[g][c] = mfma16x16x4(a[u][g], b[u][c], acc[g][c]);
                };
                load(0, a0, b0);
                for (int ch = 0; ch < nch; ch += 2) {
                    load(min(ch + 1, nch - 1), a1, b1);
                    mma(a0, b0);
                    if (ch + 1 >= nch) break;
                    load(min(ch + 2, nch - 1), a0, b0);
                    mma(a1, b1);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (!live[g]) continue;
#pragma unroll
                for (int c = 0; c < CT; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        L[(j + 16 * c + l16) * Mp + row0[g] + l4 + 4 * r] = acc[g][c][r];
            }
        }
        __syncthreads();
        // 2. factorise the diagonal block in LDS: step c reads column c of D
        //    and writes only columns > c of D and column c of Lc
        for (int e = tid; e < NB * NB; e += 256) {
            const int r = e % NB, c = e / NB;
            D[e] = r >= c ? L[(int64_t)(j + c) * Mp + j + r] : 0.0;
        }
        __syncthreads();
        for (int c = 0; c < NB; ++c) {
            const double dcc = D[c * NB + c];
            if (tid == 0 && !(dcc > 0.0)) bad = 1;
            const double s = sqrt(dcc > 0.0 ? dcc : 1.0), inv = 1.0 / s, inv2 = inv * inv;
            if (tid < NB) Lc[c * NB + tid] = tid > c ? D[c * NB + tid] * inv : (tid == c ? s : 0.0);
            if (tid == 0) Li[c] = inv;
            // lane (r, first column): rows by lane % NB, columns by lane / NB
            // in rounds of 256 / NB (no division by a run-time count)
            {
                const int r = tid % NB;
                for (int cc = c + 1 + tid / NB; cc < NB; cc += 256 / NB)
                    if (r >= cc) D[cc * NB + r] -= D[c * NB + r] * D[c * NB + cc] * inv2;
            }
            __syncthreads();
        }
        // 3. W = L11^-1, column k by thread k, built in place in LDS
        if (tid < NB) {
            const int k = tid;
            for (int i = 0; i < k; ++i) W[k * NB + i] = 0.0;
            W[k * NB + k] = Li[k];
            for (int i = k + 1; i < NB; ++i) {
                double v = 0.0;
                for (int mm = k; mm < i; ++mm) v -= Lc[mm * NB + i] * W[k * NB + mm];
                W[k * NB + i] = v * Li[i];
            }
        }
        __syncthreads();
        for (int e = tid; e < NB * NB; e += 256) {
            const int r = e % NB, c = e / NB;
            L[(int64_t)(j + c) * Mp + j + r] = Lc[e];
            Dinv[(int64_t)j * NB + e] = W[e];
        }
        // 4. rows below the diagonal block: x L11^T = a, i.e. X = A W^T, on
        //    matrix cores (A operand from the panel, B operand W^T from LDS)
        {
            const int RT4 = (Mp - j - NB) / 16;
            for (int pass = 0; pass * 4 * G < RT4; ++pass) {
                dbl4 acc[G][CT];
                int row0[G];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int t = pass * 4 * G + g * 4 + wave;
                    row0[g] = t < RT4 ? j + NB + 16 * t : -1;
#pragma unroll
                    for (int c = 0; c < CT; ++c) acc[g][c] = dbl4{0.0, 0.0, 0.0, 0.0};
                }
#pragma unroll
                for (int k0 = 0; k0 < NB; k0 += 4) {
                    double b[CT];
#pragma unroll
                    for (int c = 0; c < CT; ++c) b[c] = W[(k0 + l4) * NB + 16 * c + l16];
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        if (row0[g] < 0) continue;  // wave-uniform
                        const double a = L[(j + k0 + l4) * Mp + row0[g] + l16];
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
                        for (int r = 0; r < 4; ++r) L[(j + 16 * c + l16) * Mp + row0[g] + l4 + 4 * r] = acc[g][c][r];
                }
            }
        }
        // 5. zero the panel's columns above the diagonal block
        for (int c = 0; c < NB; ++c)
            for (int r = tid; r < j; r += 256) L[(int64_t)(j + c) * Mp + r] = 0.0;
        __syncthreads();
    }
    if (tid == 0 && bad) atomicOr(it.w.flag, 4);
}

// ---------------------------------------------------------------------------
// blocked substitutions with R right-hand sides held in LDS (row-major
// Mp x R).  Dj: NB x NB staging, T: NB x R.
// ---------------------------------------------------------------------------

// X <- L^-1 X
template <int NB, int R>
__device__ void forward_rl(const gmem<const double> L, const gmem<const double> Dinv, int Mp, double *X,
                           double *Dj, double *T) {
    const int tid = threadIdx.x;
    for (int j = 0; j < Mp; j += NB) {
        for (int e = tid; e < NB * NB; e += 256) Dj[e] = Dinv[(int64_t)j * NB + e];
        __syncthreads();
        // x_j = Dinv_j b_j
        for (int o = tid; o < NB * R; o += 256) {
            const int r = o / R, c = o % R;
            double acc = 0.0;
            for (int l = 0; l <= r; ++l) acc += Dj[l * NB + r] * X[(j + l) * R + c];
            T[o] = acc;
        }
        __syncthreads();
        for (int o = tid; o < NB * R; o += 256) X[j * R + o] = T[o];
        __syncthreads();
        // later rows: b[r] -= L[r, j:j+NB] x_j
        for (int r = j + NB + tid; r < Mp; r += 256) {
            double acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = 0.0;
#pragma unroll
            for (int l = 0; l < NB; ++l) {
                const double lv = L[(int64_t)(j + l) * Mp + r];
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] += lv * X[(j + l) * R + c];
            }
#pragma unroll
            for (int c = 0; c < R; ++c) X[r * R + c] -= acc[c];
        }
        __syncthreads();
    }
}

// X <- L^-T X
template <int NB, int R>
__device__ void backward_rl(const gmem<const double> L, const gmem<const double> Dinv, int Mp, double *X,
                            double *Dj, double *T) {
    const int tid = threadIdx.x;
    for (int j = Mp - NB; j >= 0; j -= NB) {
        for (int e = tid; e < NB * NB; e += 256) Dj[e] = Dinv[(int64_t)j * NB + e];
        __syncthreads();
        // x_j = Dinv_j^T b_j: x[r] = sum_{l >= r} Dinv_j[l][r] b[l]
        for (int o = tid; o < NB * R; o += 256) {
            const int r = o / R, c = o % R;
            double acc = 0.0;
            for (int l = r; l < NB; ++l) acc += Dj[r * NB + l] * X[(j + l) * R + c];
            T[o] = acc;
        }
        __syncthreads();
        for (int o = tid; o < NB * R; o += 256) X[j * R + o] = T[o];
        __syncthreads();
        // earlier rows: b[k] -= sum_l L[j+l][k] x[j+l]
        for (int k = tid; k < j; k += 256) {
            double acc[R];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = 0.0;
            const gmem<const double> col = L + (int64_t)k * Mp + j;
#pragma unroll
            for (int l = 0; l < NB; ++l) {
                const double lv = col[l];
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] += lv * X[(j + l) * R + c];
            }
#pragma unroll
            for (int c = 0; c < R; ++c) X[k * R + c] -= acc[c];
        }
        __syncthreads();
    }
}

// Y = L^-1 K_p, S = Y^T Y, Sc = chol(S); one workgroup per body.
template <int NB>
__global__ __launch_bounds__(256) void project_large_kernel(const BigBody *__restrict__ items) {
    extern __shared__ double lds[];
    __shared__ double Dj[NB * NB];
    __shared__ double T[NB * 6];
    __shared__ double S[36];
    __shared__ int bad;
    const BigBody it = items[blockIdx.x];
    const int Mp = it.Mp, m = 3 * it.w.n_blobs, tid = threadIdx.x;
    const gmem<const double> L = as_global(it.w.factor);
    double *Y = lds;  // Mp x 6
    if (tid == 0) bad = 0;
    const gmem<const double> q = as_global(it.w.q);
    for (int e = tid; e < 6 * Mp; e += 256) {
        const int row = e / 6, k = e % 6;
        double v = 0.0;
        if (row < m) {
            const int i = row / 3, c = row % 3;
            const gmem<const double> ri = as_global(it.w.pos + 3 * (it.w.blob0 + i));
            const double d[3] = {ri[0] - q[0], ri[1] - q[1], ri[2] - q[2]};
            v = K_entry(d, c, k);
        }
        Y[e] = v;
    }
    __syncthreads();
    forward_rl<NB, 6>(L, as_global((const double *)big_Dinv(it)), Mp, Y, Dj, T);
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
    double *Yg = big_Y(it);
    for (int e = tid; e < 6 * Mp; e += 256) as_global(Yg)[e] = Y[e];
    double *Sc = big_Sc(it);
    if (tid < 36) as_global(Sc)[tid] = ((tid % 6) <= (tid / 6)) ? S[tid] : 0.0;
    if (tid == 0 && bad) atomicOr(it.w.flag, 8);
}

// Apply P^-1 to up to 8 right-hand sides of one body per workgroup
// (grid.y = groups of 8 rhs).  lds: X (Mp x 8).
template <int NB>
__global__ __launch_bounds__(256) void apply_large_kernel(const PrecondApplyJob *__restrict__ jobs, int32_t n_jobs) {
    constexpr int R = 8, QP = 16;  // rhs per workgroup; partial sums per (rhs, k) of Y^T t
    extern __shared__ double lds[];
    __shared__ double Dj[NB * NB > QP * R * 6 ? NB * NB : QP * R * 6];
    __shared__ double T[NB * R];
    __shared__ double g[R][6];
    const int64_t w = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= w) lo = mid; else hi = mid - 1;
    }
    const PrecondApplyJob &J = jobs[lo];
    const BigBody it = ((const BigBody *)J.items)[w - J.wg_begin];
    const int Mp = it.Mp, m = 3 * it.w.n_blobs, tid = threadIdx.x;
    const int r0 = R * blockIdx.y;
    const int nr = min(R, J.nrhs - r0);
    if (nr <= 0) return;
    const gmem<const double> L = as_global(it.w.factor);
    const double *Y = big_Y(it), *Dinv = big_Dinv(it), *Sc = big_Sc(it);
    double *X = lds;  // Mp x 8
    const bool resist = J.mode != 0;  // resistance problem: lambda = M_pp^-1 s only
    const int64_t b3 = 3 * it.w.blob0, u6 = resist ? 0 : J.nb3 + 6 * (int64_t)it.w.body;
    // with a shared reference-shape factor, the right-hand sides are taken
    // into the body frame (R^T on every 3-vector) and the results back (R)
    const gmem<const double> Rot = as_global(it.w.rot);
    if (it.w.rot) {
        for (int e = tid; e < Mp * R; e += 256) {
            const int row = e / R, c = e % R;
            double v = 0.0;
            if (row < m && c < nr) {
                const gmem<const double> x = as_global(J.in) + (int64_t)(r0 + c) * J.ld + b3 + row - row % 3;
                const int k = row % 3;
                v = Rot[k] * x[0] + Rot[3 + k] * x[1] + Rot[6 + k] * x[2];
            }
            X[e] = v;
        }
    } else {
        for (int e = tid; e < Mp * R; e += 256) {
            const int row = e / R, c = e % R;
            X[e] = (row < m && c < nr) ? as_global(J.in)[(int64_t)(r0 + c) * J.ld + b3 + row] : 0.0;
        }
    }
    __syncthreads();
    forward_rl<NB, R>(L, as_global(Dinv), Mp, X, Dj, T);
    if (!resist) {
        // g = F - Y^T t, F = -bottom: thread (c, qp) sums rows l = qp (mod QP)
        // for k = 0..5, then the QP partials are added in order
        double *part = Dj;  // [QP][R][6]
        if (tid < QP * R) {
            const int c = tid % R, qp = tid / R;
            double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
            for (int l = qp; l < Mp; l += QP) {
                const double x = X[l * R + c];
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[k] += as_global(Y)[l * 6 + k] * x;
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) part[(qp * R + c) * 6 + k] = acc[k];
        }
        __syncthreads();
        if (tid < R * 6) {
            const int c = tid / 6, k = tid % 6;
            double acc = 0.0;
            for (int qp = 0; qp < QP; ++qp) acc += part[(qp * R + c) * 6 + k];
            double bot = 0.0;
            if (c < nr) {
                const gmem<const double> x = as_global(J.in) + (int64_t)(r0 + c) * J.ld + u6;
                if (it.w.rot) {
                    const int b = k - k % 3, kk = k % 3;
                    bot = Rot[kk] * x[b] + Rot[3 + kk] * x[b + 1] + Rot[6 + kk] * x[b + 2];
                } else {
                    bot = x[k];
                }
            }
            g[c][k] = c < nr ? -bot - acc : 0.0;
        }
        __syncthreads();
        if (tid < nr) {
            double u[6];
            double *gg = g[tid];
            for (int i = 0; i < 6; ++i) {
                double v = gg[i];
                for (int k = 0; k < i; ++k) v -= as_global(Sc)[i * 6 + k] * u[k];
                u[i] = v / as_global(Sc)[i * 6 + i];
            }
            for (int i = 5; i >= 0; --i) {
                double v = u[i];
                for (int k = i + 1; k < 6; ++k) v -= as_global(Sc)[k * 6 + i] * gg[k];
                gg[i] = v / as_global(Sc)[i * 6 + i];
            }
        }
        __syncthreads();
        for (int row = tid; row < Mp; row += 256) {
            double yk[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) yk[k] = as_global(Y)[row * 6 + k];
#pragma unroll
            for (int c = 0; c < R; ++c) {
                double acc = X[row * R + c];
#pragma unroll
                for (int k = 0; k < 6; ++k) acc += yk[k] * g[c][k];
                X[row * R + c] = acc;
            }
        }
        __syncthreads();
    }
    backward_rl<NB, R>(L, as_global(Dinv), Mp, X, Dj, T);
    if (it.w.rot) {
        // backward_rl ends with a barrier, so all of X is final here
        for (int e = tid; e < m * R; e += 256) {
            const int row = e / R, c = e % R;
            if (c < nr) {
                const int b = row - row % 3, k = row % 3;
                as_global(J.out)[(int64_t)(r0 + c) * J.ld + b3 + row] =
                    Rot[3 * k] * X[b * R + c] + Rot[3 * k + 1] * X[(b + 1) * R + c] + Rot[3 * k + 2] * X[(b + 2) * R + c];
            }
        }
        if (tid < R * 6 && !resist) {
            const int c = tid / 6, k = tid % 6;
            const int b = k - k % 3, kk = k % 3;
            if (c < nr)
                as_global(J.out)[(int64_t)(r0 + c) * J.ld + u6 + k] =
                    Rot[3 * kk] * g[c][b] + Rot[3 * kk + 1] * g[c][b + 1] + Rot[3 * kk + 2] * g[c][b + 2];
        }
        return;
    }
    for (int e = tid; e < m * R; e += 256) {
        const int row = e / R, c = e % R;
        if (c < nr) as_global(J.out)[(int64_t)(r0 + c) * J.ld + b3 + row] = X[e];
    }
    if (tid < R * 6 && !resist) {
        const int c = tid / 6, k = tid % 6;
        if (c < nr) as_global(J.out)[(int64_t)(r0 + c) * J.ld + u6 + k] = g[c][k];
    }
}

// ---------------------------------------------------------------------------

// Tile shapes the autotuner times: {panel width, row tiles per wave, steps
// per prefetched chunk}.  Shapes with G * U <= 8 stay within 256 VGPRs
// (two bodies per CU); the others trade occupancy for operand reuse.
struct LargeShape {
    int nb, g, u;
};
static constexpr LargeShape kLargeShapes[] = {{16, 2, 4}, {32, 2, 4}, {32, 2, 8}, {32, 4, 2}, {32, 1, 8}, {16, 4, 4}};
constexpr int kLargeVariants = (int)(sizeof(kLargeShapes) / sizeof(kLargeShapes[0]));

int large_variant_count() { return kLargeVariants; }
int large_panel_width(int variant) { return kLargeShapes[variant].nb; }
void large_variant_shape(int variant, int *nb, int *row_tiles, int *chunk) {
    *nb = kLargeShapes[variant].nb;
    *row_tiles = kLargeShapes[variant].g;
    *chunk = 4 * kLargeShapes[variant].u;
}

template <int V>
static void launch_chol(const BigBody *items, int32_t n_items, hipStream_t s) {
    constexpr LargeShape sh = kLargeShapes[V];
    hipLaunchKernelGGL((chol_large_kernel<sh.nb, sh.g, sh.u>), dim3(n_items), dim3(256), 0, s, items);
}

hipError_t launch_precond_build_large(const BigBody *items, int32_t n_items, int max_Mp, int variant, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (variant < 0 || variant >= kLargeVariants) return hipErrorInvalidValue;
    hipLaunchKernelGGL(assemble_large_kernel, dim3(n_items, asm_tiles(max_Mp)), dim3(256), 0, s, items);
    switch (variant) {
        case 0: launch_chol<0>(items, n_items, s); break;
        case 1: launch_chol<1>(items, n_items, s); break;
        case 2: launch_chol<2>(items, n_items, s); break;
        case 3: launch_chol<3>(items, n_items, s); break;
        case 4: launch_chol<4>(items, n_items, s); break;
        default: launch_chol<5>(items, n_items, s); break;
    }
    static_assert(kLargeVariants == 6, "launch switch covers every shape");
    const size_t lds = (size_t)max_Mp * 6 * sizeof(double);
    if (large_panel_width(variant) == 32)
        hipLaunchKernelGGL(project_large_kernel<32>, dim3(n_items), dim3(256), lds, s, items);
    else
        hipLaunchKernelGGL(project_large_kernel<16>, dim3(n_items), dim3(256), lds, s, items);
    return hipGetLastError();
}

hipError_t launch_precond_apply_large(const PrecondApplyJob *jobs, int32_t n_jobs, int64_t n_wg, int32_t max_rhs,
                                      int max_Mp, int panel, hipStream_t s) {
    if (n_wg <= 0 || max_rhs <= 0) return hipSuccess;
    const size_t lds = (size_t)max_Mp * 8 * sizeof(double);
    dim3 g((unsigned)n_wg, (max_rhs + 7) / 8);
    if (panel != 16 && panel != 32) return hipErrorInvalidValue;
    if (panel == 32)
        hipLaunchKernelGGL(apply_large_kernel<32>, g, dim3(256), lds, s, jobs, n_jobs);
    else
        hipLaunchKernelGGL(apply_large_kernel<16>, g, dim3(256), lds, s, jobs, n_jobs);
    return hipGetLastError();
}

}  // namespace rmb

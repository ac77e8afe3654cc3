// Preconditioner build and apply for bodies whose 3n x 3n mobility block is
// too large for LDS (Sec. 2.2.2: the per-body factorisation of M_pp behind
// eq:saddle_M_precon), e.g. 162-blob shells (486 x 486).
//
// Storage per body (doubles), Mp = 3n + 6 rounded up to 64; rows and
// columns past 3n hold the identity, so the padded factor is blockdiag(L, I)
// (rows 3n .. 3n+5 carry K_p^T while the block is factorised):
//   L    : Mp x Mp, column-major, lower triangle (the upper triangle is zero)
//   Y    : Mp x 6, row-major (L^-1 K_p, zero in the padding)
//   Dinv : the inverses of L's NB x NB diagonal blocks, block j/NB at
//          offset j*NB, each column-major (room for NB = 32: Mp x 32)
//   Sc   : 6 x 6 lower (Cholesky factor of S = Y^T Y)
//
// Build, two launches covering all bodies: assembly of the lower triangle
// (with the bordered rows), then the factorisation, which yields L, the
// diagonal-block inverses, Y, S and Sc.
//
// Cholesky: one workgroup (4 waves) per body, left-looking by panels of 64
// columns.  Panel update
//   A[j:, j:j+64] -= L[j:, 0:j] L[j:j+64, 0:j]^T
// runs on FP64 matrix cores (v_mfma_f64_16x16x4: D[16x16] += A[16x4] B[4x16]);
// the operands of the next chunk of columns of L are loaded while the
// current ones are multiplied.  The panel's diagonal block is updated first,
// factorised in LDS and inverted; then the rows below are updated pass by
// pass and, still in registers, become x = a L11^-T, a product with the
// inverse, also on matrix cores, so each element of L is stored once.
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
    // rows m..Mp-1 of columns 0..m-1: the border K_p^T (rows m..m+5), then zero
    const int64_t padr = (int64_t)(Mp - m) * m;
    const gmem<const double> q = as_global(it.w.q);
    for (int64_t e = (int64_t)g * 256 + tid; e < padr; e += stride) {
        const int64_t col = e / (Mp - m), row = m + e % (Mp - m);
        double v = 0.0;
        if (row < m + 6) {
            const int i = (int)(col / 3), c = (int)(col % 3);
            const gmem<const double> ri = as_global(it.w.pos + 3 * (it.w.blob0 + i));
            const double d[3] = {ri[0] - q[0], ri[1] - q[1], ri[2] - q[2]};
            v = K_entry(d, c, (int)(row - m));
        }
        A[col * Mp + row] = v;
    }
}

// ---------------------------------------------------------------------------
// left-looking blocked Cholesky, panels of 64 columns, FP64 matrix cores
// ---------------------------------------------------------------------------

constexpr int kPanel = 64;
constexpr int kLd = kPanel + 2;  // LDS leading dimension of the diagonal block: rows in other banks

// Operand loads of the factorisation go through a buffer resource: the
// per-lane part of an address is a 32-bit offset fixed for a whole pass,
// the part that moves with the column is a wave-uniform (scalar) offset, so
// a prefetched chunk costs no 64-bit address registers.
typedef __amdgpu_buffer_rsrc_t brsrc;
__device__ __forceinline__ brsrc factor_rsrc(const BigBody &it) {
    return __builtin_amdgcn_make_buffer_rsrc(it.w.factor, (short)0, (int)((int64_t)it.Mp * it.Mp * 8), 0x00020000);
}
__device__ __forceinline__ double bload(brsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(double v, brsrc r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned int, v), r,
                                          voff, soff, 0);
}

// LDS of one workgroup.  W, the inverse of the panel's diagonal block, lives
// from its factorisation through the panel's row solve; the rest is shared
// by phases that never overlap: the block itself while it is factorised, the
// staged B chunks of an update pass, the per-wave transposes of the row
// solve (after the pass's last chunk), and the bordered rows at the end.
constexpr int kXld = 17;  // leading dimension of a transposed 16 x 64 tile
struct CholLds {
    double W[kPanel * kLd];  // column-major (leading dimension kLd)
    union {
        struct {
            double D[kPanel * kLd];  // diagonal block, column-major (leading dimension kLd)
            double T[4][16 * 16];    // per wave: a 16 x 16 product, column-major
        } d;
        double B[2][32 * kPanel];    // chunk of L[j:j+64, k0:k0+KC], column-major (KC <= 32)
        double X[4][kPanel * kXld];  // per wave: a 16 x 64 tile, column-major
        double Yt[6 * 768];          // epilogue: the bordered rows (Y^T), row k at k * m
    };
    double rdiag[kPanel];  // 1 / L[c][c] of the block (1 in the padding)
    double S[36];
    int bad;
};

// 1 / sqrt(x) for x > 0: the hardware estimate and one third-order
// correction step, y (1 + e/2 + 3e^2/8) with e = 1 - x y^2.
__device__ __forceinline__ double rsqrt64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

// Lanes of one wave exchange a double through two readlanes (the lane index
// is a constant, so the value lands in scalar registers).
__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// LDS ordering inside one wave: the wave's earlier LDS writes are complete
// before its later reads (other lanes' values), and the compiler keeps the
// order.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// 16 x 16 tiles in LDS, column-major with leading dimension ld (element (i, j)
// at P[j * ld + i]), on the matrix cores.  C layout: lane holds rows
// l4 + 4 r, column l16.
__device__ __forceinline__ dbl4 tile_load(const double *P, int ld, int l16, int l4) {
    return dbl4{P[l16 * ld + l4], P[l16 * ld + l4 + 4], P[l16 * ld + l4 + 8], P[l16 * ld + l4 + 12]};
}
__device__ __forceinline__ void tile_store(double *P, int ld, int l16, int l4, dbl4 v) {
#pragma unroll
    for (int r = 0; r < 4; ++r) P[l16 * ld + l4 + 4 * r] = v[r];
}
// acc += sA * A B with A (16 x 16) and B (16 x 16) column-major tiles; with
// TB, B is given as its transpose (B[k][n] = Bt[n][k]).
template <bool TB>
__device__ __forceinline__ dbl4 tile_mma(dbl4 acc, const double *A, int lda, const double *B, int ldb, double sA,
                                         int l16, int l4) {
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
        const double a = sA * A[(k0 + l4) * lda + l16];
        const double b = TB ? B[(k0 + l4) * ldb + l16] : B[l16 * ldb + k0 + l4];
        acc = mfma16x16x4(a, b, acc);
    }
    return acc;
}

// Update of row tiles of panel j (columns [j, j + 64)) by the columns [0, j)
// to its left,
//   A[r, j:j+64] -= L[r, 0:j] L[j:j+64, 0:j]^T,
// wave w taking tiles tb + w + 4 g, g < G, of rows [j, Mp) (clamped at the
// last tile: a clamped tile does no arithmetic, live[g] false).  The B
// operand L[j:j+64, k0:k0+KC] is staged in LDS per chunk of KC columns
// (double buffered, one barrier per chunk), the A operand is read straight
// from the factor, a chunk ahead.  The accumulators start at -A and take
// +L L^T, so no operand needs a sign change: acc[g] ends as minus the
// updated tile, lane holding rows l4 + 4 r, column 16 c + l16 in
// acc[g][c][r], and vod[g] is the byte offset of that lane's element
// (row l4, column l16) of the tile.  With j = 0 the tiles are just loaded.
template <int G, int KC>
__device__ __forceinline__ void update_tiles(brsrc rs, int Mp, int j, int tb, dbl4 (&acc)[G][4], bool (&live)[G],
                                             uint32_t (&vod)[G], CholLds &sh) {
    constexpr int KS = KC / 4;  // MFMA steps per chunk
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const int RT = (Mp - j) / 16;
    const int nch = j / KC;
    const uint32_t colb = (uint32_t)Mp * 8;  // bytes per column of L
    int row0[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int t = tb + g * 4 + wave;
        live[g] = __builtin_amdgcn_readfirstlane(t < RT ? 1 : 0) != 0;  // wave-uniform: a scalar branch
        row0[g] = j + 16 * (t < RT ? t : RT - 1);  // clamped: loads stay unconditional
        vod[g] = ((uint32_t)(j + l16) * Mp + row0[g] + l4) * 8;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[g][c][r] = -bload(rs, vod[g], (16 * c) * colb + 32 * r);
    }
    if (nch == 0) return;
    // B staging: thread tid loads KC * 64 / 256 values of the chunk
    constexpr int BV = KC * kPanel / 256;
    double bst[BV];
    double a0[KS][G], a1[KS][G];
    uint32_t voa[G];
#pragma unroll
    for (int g = 0; g < G; ++g) voa[g] = ((uint32_t)l4 * Mp + row0[g] + l16) * 8;
    const uint32_t vob = ((uint32_t)(tid / kPanel) * Mp + j + tid % kPanel) * 8;  // + v * (256 / 64) columns
    auto load_b = [&](int ch) {
#pragma unroll
        for (int v = 0; v < BV; ++v) bst[v] = bload(rs, vob, (uint32_t)(ch * KC + v * (256 / kPanel)) * colb);
    };
    auto put_b = [&](int buf) {
#pragma unroll
        for (int v = 0; v < BV; ++v) sh.B[buf][tid + 256 * v] = bst[v];
    };
    auto load_a = [&](int ch, double (&a)[KS][G]) {
#pragma unroll
        for (int u = 0; u < KS; ++u)
#pragma unroll
            for (int g = 0; g < G; ++g) a[u][g] = bload(rs, voa[g], (uint32_t)(ch * KC + 4 * u) * colb);
    };
    auto mma = [&](int buf, const double (&a)[KS][G]) {
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            double b[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = sh.B[buf][(4 * u + l4) * kPanel + 16 * c + l16];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (!live[g]) continue;  // wave-uniform: a clamped tile does no arithmetic
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[g][c] = mfma16x16x4(a[u][g], b[c], acc[g][c]);
            }
        }
    };
    // The prefetches are unconditional (the chunk index is clamped at the
    // last chunk): with no branch around them the compiler counts exactly
    // how many loads are in flight behind each operand and waits for that
    // one only.
    load_b(0);
    load_a(0, a0);
    __syncthreads();  // the previous phase is done with the LDS
    put_b(0);
    for (int ch = 0; ch < nch; ch += 2) {
        // chunk ch in buffer 0 / registers a0; chunk ch + 1 loaded meanwhile
        load_b(min(ch + 1, nch - 1)), load_a(min(ch + 1, nch - 1), a1);
        __syncthreads();
        mma(0, a0);
        if (ch + 1 >= nch) break;
        put_b(1);
        load_b(min(ch + 2, nch - 1)), load_a(min(ch + 2, nch - 1), a0);
        __syncthreads();
        mma(1, a1);
        put_b(0);  // every wave is past mma(0): buffer 0 is free
    }
}

// The panel's diagonal block, updated, into LDS:
//   D = A[j:j+64, j:j+64] - L[j:j+64, 0:j] L[j:j+64, 0:j]^T,
// its lower 16 x 16 tiles only (the upper ones are left as they are and
// never read).  The k range of the product is split over the waves (wave w
// takes columns [w j/4, (w+1) j/4)), and one set of loads serves as both
// operands, since both are rows of L[j:j+64, 0:j]; the next step's operands
// are loaded while the current ones are multiplied.  Then wave 0 stores A
// minus its sum and each further wave subtracts its own, in wave order.
__device__ __forceinline__ void diag_rows(brsrc rs, int Mp, int j, CholLds &sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    double *D = sh.d.D;
    const uint32_t colb = (uint32_t)Mp * 8;  // bytes per column of L
    dbl4 acc[10];                            // tile (t, c), c <= t, at t (t + 1) / 2 + c
#pragma unroll
    for (int i = 0; i < 10; ++i) acc[i] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int kq = j / 4;  // a multiple of 16
    const int k0 = wave * kq, k1 = k0 + kq;
    uint32_t vo[4];  // lane's element (row j + 16 t + l16, column l4)
#pragma unroll
    for (int t = 0; t < 4; ++t) vo[t] = ((uint32_t)l4 * Mp + j + 16 * t + l16) * 8;
    auto load = [&](int k, double (&v)[4]) {
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = bload(rs, vo[t], (uint32_t)k * colb);
    };
    auto mma = [&](const double (&v)[4]) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int c = 0; c <= t; ++c) acc[t * (t + 1) / 2 + c] = mfma16x16x4(v[t], v[c], acc[t * (t + 1) / 2 + c]);
    };
    if (kq > 0) {
        double v0[4], v1[4];
        load(k0, v0);
        for (int k = k0; k < k1; k += 8) {
            load(k + 4, v1);  // kq is a multiple of 8: k + 4 < k1
            mma(v0);
            load(min(k + 8, k1 - 4), v0);  // clamped on the last step (loaded, not used)
            mma(v1);
        }
    }
    for (int w = 0; w < 4; ++w) {
        if (w > 0 && kq == 0) break;  // uniform: nothing to subtract
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int c = 0; c <= t; ++c) {
                    double *C = D + (16 * c) * kLd + 16 * t;
                    dbl4 x;
                    if (w == 0) {
                        const uint32_t va = ((uint32_t)(j + 16 * c + l16) * Mp + j + 16 * t + l4) * 8;
#pragma unroll
                        for (int r = 0; r < 4; ++r) x[r] = bload(rs, va, 32 * r);
                    } else {
                        x = tile_load(C, kLd, l16, l4);
                    }
                    tile_store(C, kLd, l16, l4, x - acc[t * (t + 1) / 2 + c]);
                }
        }
        __syncthreads();
    }
}

// One workgroup (4 waves) per body, all bodies in one launch.  The factored
// matrix is [M_pp; K_p^T] bordered below by the 6 rows of K_p^T (rows m ..
// m+5 of the padded block, written by the assembly): its Cholesky rows there
// are K_p^T L^-T = Y^T, so the factorisation yields Y = L^-1 K_p as well;
// only the first m columns are factorised (the others are padding, kept at
// the identity).  Per panel of 64 columns:
//   1. the panel's diagonal block, updated on matrix cores (diag_rows), to
//      LDS;
//   2. its Cholesky factor and inverse W (diag_block);
//   3. the rows below, in passes of row tiles: each tile updated, then
//      solved in registers, X = A W^T, on matrix cores, and stored once.
// At the end Y^T is moved from the bordered rows into the Y storage,
// S = Y^T Y and its Cholesky factor are formed, and the bordered rows are
// cleared so that the stored L is blockdiag(L, I).
//
// Step 2: the 64 x 64 diagonal block in LDS is factorised (its L written to
// the factor at columns [j, j+64)) and inverted into W.  A function of its
// own so that its registers are allocated apart from the matrix-core
// phases'.
__device__ __attribute__((noinline)) void diag_block(gmem<double> L, int Mp, int j, int m, CholLds &sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    double *D = sh.d.D, *W = sh.W;
    // 2. the 64 x 64 diagonal block in LDS, factorised in four column
    //    blocks of 16: wave b factorises block b alone (lane = row, the
    //    block's 16 columns in registers, values shared by readlane, no
    //    barrier), then the waves to its right take its rank-16 update
    //    on the matrix cores.  Columns [0, nc) are the matrix's, the
    //    rest padding (the identity).
    const int nc = max(0, min(kPanel, m - j));
    // unrolled: every readlane below takes a constant lane
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (wave == b) {
            const int r = lane;
            double d[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) d[c] = D[(16 * b + c) * kLd + r];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int C = 16 * b + c;
                if (C < nc) {  // uniform
                    const double dcc = lane_value(d[c], C);
                    const double inv = rsqrt64(dcc > 0.0 ? dcc : 1.0);
                    if (lane == 0) {
                        sh.rdiag[C] = inv;
                        if (!(dcc > 0.0)) sh.bad = 1;
                    }
                    d[c] = r >= C ? d[c] * inv : 0.0;
                    // rows above a later column's diagonal take the update
                    // too; they are cleared when that column is finished
#pragma unroll
                    for (int k = c + 1; k < 16; ++k) d[k] -= d[c] * lane_value(d[c], 16 * b + k);
                } else {
                    d[c] = r == C ? 1.0 : 0.0;
                    if (lane == 0) sh.rdiag[C] = 1.0;
                }
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) D[(16 * b + c) * kLd + r] = d[c];
        }
        __syncthreads();
        if (wave > b) {
            // D[16t.., 16w..] -= L[16t.., 16b..] L[16w.., 16b..]^T for row tiles t >= w
            for (int t = wave; t < 4; ++t) {
                double *C = D + (16 * wave) * kLd + 16 * t;
                dbl4 acc = tile_load(C, kLd, l16, l4);
                acc = tile_mma<true>(acc, D + (16 * b) * kLd + 16 * t, kLd, D + (16 * b) * kLd + 16 * wave, kLd, -1.0,
                                     l16, l4);
                tile_store(C, kLd, l16, l4, acc);
            }
        }
        __syncthreads();
    }
    // the factor's block to global memory (the upper part as zeros,
    // bordered rows included); in LDS the rows from m on (border or
    // padding) and the upper part are cleared: the block to invert
    for (int e = tid; e < kPanel * kPanel; e += 256) {
        const int r = e % kPanel, c = e / kPanel;
        double v = D[c * kLd + r];
        if (r < c) v = 0.0;
        L[(j + c) * Mp + j + r] = v;
        if ((j + r >= m && c < nc) || r < c) D[c * kLd + r] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    // W = D^-1 by blocks of 16: each wave inverts its diagonal block
    // (lane k < 16 holds column k, forward substitution), then wave j
    // forms its block column below, X_ij = -W_ii sum_{j <= k < i} L_ik X_kj
    {
        const int w16 = 16 * wave;
        if (lane < 16) {
            const int k = lane;
            double x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                double v = i == k ? 1.0 : 0.0;
#pragma unroll
                for (int q = 0; q < i; ++q) v -= D[(w16 + q) * kLd + w16 + i] * x[q];
                x[i] = i >= k ? v * sh.rdiag[w16 + i] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) W[(w16 + k) * kLd + w16 + i] = x[i];
        }
        // blocks above the diagonal are zero
        for (int e = lane; e < 16 * w16; e += 64) W[(w16 + e / w16) * kLd + e % w16] = 0.0;
    }
    __syncthreads();
    {
        const int jb = wave;  // block column
        double *T = sh.d.T[wave];
        for (int i = jb + 1; i < 4; ++i) {
            dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
            for (int k = jb; k < i; ++k)
                acc = tile_mma<false>(acc, D + (16 * k) * kLd + 16 * i, kLd, W + (16 * jb) * kLd + 16 * k, kLd, 1.0,
                                      l16, l4);
            tile_store(T, 16, l16, l4, acc);
            wave_lds_sync();
            acc = tile_mma<false>(dbl4{0.0, 0.0, 0.0, 0.0}, W + (16 * i) * kLd + 16 * i, kLd, T, 16, -1.0, l16, l4);
            tile_store(W + (16 * jb) * kLd + 16 * i, kLd, l16, l4, acc);
            wave_lds_sync();
        }
    }
    __syncthreads();
}

template <int G, int KC>
__global__ __launch_bounds__(256, 2) void chol_panel_kernel(const BigBody *__restrict__ items) {
    __shared__ CholLds sh;
    const BigBody it = items[blockIdx.x];
    const int Mp = it.Mp, m = 3 * it.w.n_blobs;
    const gmem<double> L = as_global(it.w.factor);
    const gmem<double> Dinv = as_global(big_Dinv(it));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const uint32_t colb = (uint32_t)Mp * 8;  // bytes per column of L
    const brsrc rs = factor_rsrc(it);
    if (tid == 0) sh.bad = 0;

    for (int j = 0; j < Mp; j += kPanel) {
        const int RT = (Mp - j) / 16;
        diag_rows(rs, Mp, j, sh);  // 1. (ends with a barrier)
        diag_block(L, Mp, j, m, sh);
        const int nc = max(0, min(kPanel, m - j));
        // stored inverses of the two 32 x 32 diagonal blocks (the substitutions' blocks)
        for (int e = tid; e < 2 * 32 * 32; e += 256) {
            const int b = e / 1024, o = e % 1024, r = o % 32, c = o / 32;
            Dinv[(int64_t)(j + 32 * b) * 32 + o] = sh.W[(32 * b + c) * kLd + 32 * b + r];
        }
        // 3. the rows below, 4G tiles per pass: each tile updated, then
        //    X = A W^T with A from the accumulators (through a per-wave
        //    transpose in LDS) and B = W^T from LDS; columns past m are zero.
        //    Every element of L below the diagonal block is stored once.
        for (int tb = 4; tb < RT; tb += 4 * G) {
            dbl4 acc[G][4];
            bool live[G];
            uint32_t vod[G];
            update_tiles<G, KC>(rs, Mp, j, tb, acc, live, vod, sh);
            __syncthreads();  // the staged chunks are no longer read: the transposes overlay them
            double *Xw = sh.X[wave];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (!live[g]) continue;  // wave-uniform
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) Xw[(16 * c + l16) * kXld + l4 + 4 * r] = -acc[g][c][r];
                wave_lds_sync();
                dbl4 x[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) x[c] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const double a = Xw[(4 * u + l4) * kXld + l16];
                    double b[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) b[c] = sh.W[(4 * u + l4) * kLd + 16 * c + l16];
#pragma unroll
                    for (int c = 0; c < 4; ++c) x[c] = mfma16x16x4(a, b[c], x[c]);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const bool keep = 16 * c + l16 < nc;
#pragma unroll
                    for (int r = 0; r < 4; ++r) bstore(keep ? x[c][r] : 0.0, rs, vod[g], (16 * c) * colb + 32 * r);
                }
                wave_lds_sync();  // the tile's reads are done before the next tile's writes
            }
        }
        __syncthreads();  // the next panel's phases reuse the LDS
    }

    // Y^T from the bordered rows (then cleared), S = Y^T Y, its Cholesky factor
    gmem<double> Y = as_global(big_Y(it));
    for (int e = tid; e < 6 * m; e += 256) {
        const int k = e / m, i = e % m;
        const int64_t a = (int64_t)i * Mp + m + k;
        sh.Yt[e] = L[a];
        L[a] = 0.0;
    }
    __syncthreads();
    for (int e = tid; e < 6 * Mp; e += 256) {
        const int i = e / 6, k = e % 6;
        Y[e] = i < m ? sh.Yt[k * m + i] : 0.0;
    }
    if (tid < 36) {
        // S[a][b]: a wave's lanes each take one entry, sums in index order
        const int a = tid / 6, b = tid % 6;
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += sh.Yt[a * m + i] * sh.Yt[b * m + i];
        sh.S[tid] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        double *S = sh.S;
        bool badS = false;
        for (int jj = 0; jj < 6; ++jj) {
            double dj = S[jj * 6 + jj];
            for (int k = 0; k < jj; ++k) dj -= S[jj * 6 + k] * S[jj * 6 + k];
            if (!(dj > 0.0)) badS = true, dj = 1.0;
            const double ljj = sqrt(dj);
            S[jj * 6 + jj] = ljj;
            for (int i = jj + 1; i < 6; ++i) {
                double v = S[i * 6 + jj];
                for (int k = 0; k < jj; ++k) v -= S[i * 6 + k] * S[jj * 6 + k];
                S[i * 6 + jj] = v / ljj;
            }
        }
        if (badS) atomicOr(it.w.flag, 8);
        if (sh.bad) atomicOr(it.w.flag, 4);
    }
    __syncthreads();
    if (tid < 36) as_global(big_Sc(it))[tid] = (tid % 6) <= (tid / 6) ? sh.S[tid] : 0.0;
}

// ---------------------------------------------------------------------------
// blocked substitutions with R right-hand sides held in LDS, one column of
// Mp per right-hand side (X[c * Mp + row]: threads updating consecutive rows
// touch consecutive words).  Dj: the NB x NB diagonal-block inverse staged
// with leading dimension NB + 1 (read by rows and by columns without bank
// conflicts); T: the block's solved unknowns x_j, row-major NB x R.  Per
// block: the next block's inverse and the first tile's operands of this
// block's update are loaded before they are needed (neither depends on x_j).
// ---------------------------------------------------------------------------

template <int NB>
__device__ __forceinline__ void load_dinv(const gmem<const double> Dinv, int j, double (&d)[NB * NB / 256]) {
#pragma unroll
    for (int i = 0; i < NB * NB / 256; ++i) d[i] = Dinv[(int64_t)j * NB + threadIdx.x + 256 * i];
}
template <int NB>
__device__ __forceinline__ void put_dinv(const double (&d)[NB * NB / 256], double *Dj) {
#pragma unroll
    for (int i = 0; i < NB * NB / 256; ++i) {
        const int e = threadIdx.x + 256 * i;
        Dj[(e / NB) * (NB + 1) + e % NB] = d[i];
    }
}

// X <- L^-1 X.  The later rows' update of block j,
//   X[r][c] -= sum_l L[r][j+l] x_j[l][c],  r >= j + NB,
// runs on the matrix cores, 16 rows per tile: lane (l16, l4) holds
// L[r0 + l16][j + 4s + l4] (16 consecutive words of a column across the
// lanes) as the A operand and x_j[4s + l4][l16] (zero for l16 >= R) as the B
// operand; the next tile's operands are loaded while the current one is
// multiplied.
template <int NB, int R>
__device__ void forward_rl(const gmem<const double> L, const gmem<const double> Dinv, int Mp, double *X,
                           double *Dj, double *T) {
    static_assert(NB == 32 && R <= 16, "tiles of 16 rows, 8 MFMA steps of 4 columns");
    constexpr int S = NB / 4;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    double dn[NB * NB / 256];
    load_dinv<NB>(Dinv, 0, dn);
    for (int j = 0; j < Mp; j += NB) {
        put_dinv<NB>(dn, Dj);
        const int r0 = j + NB, nt = (Mp - r0) / 16;  // row tiles below the block
        auto load_tile = [&](int t, double (&a)[S]) {
            const int64_t r = r0 + 16 * min(t, nt - 1) + l16;  // clamped: the loads stay unconditional
#pragma unroll
            for (int s = 0; s < S; ++s) a[s] = L[(int64_t)(j + 4 * s + l4) * Mp + r];
        };
        double a0[S], a1[S];
        if (nt > 0) load_tile(wave, a0);  // before the block solve: it does not depend on x_j
        __syncthreads();
        // x_j = Dinv_j b_j
        for (int o = tid; o < NB * R; o += 256) {
            const int r = o % NB, c = o / NB;
            double acc = 0.0;
            for (int l = 0; l <= r; ++l) acc += Dj[l * (NB + 1) + r] * X[c * Mp + j + l];
            T[r * R + c] = acc;
        }
        __syncthreads();
        for (int o = tid; o < NB * R; o += 256) X[(o / NB) * Mp + j + o % NB] = T[(o % NB) * R + o / NB];
        if (j + NB < Mp) load_dinv<NB>(Dinv, j + NB, dn);
        double bx[S];
#pragma unroll
        for (int s = 0; s < S; ++s) bx[s] = l16 < R ? T[(4 * s + l4) * R + l16] : 0.0;
        auto tile = [&](int t, const double (&a)[S]) {
            dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < S; ++s) acc = mfma16x16x4(a[s], bx[s], acc);
            if (l16 < R) {
#pragma unroll
                for (int r = 0; r < 4; ++r) X[l16 * Mp + r0 + 16 * t + l4 + 4 * r] -= acc[r];
            }
        };
        for (int t = wave; t < nt; t += 8) {
            load_tile(t + 4, a1);
            tile(t, a0);
            if (t + 4 >= nt) break;
            load_tile(t + 8, a0);
            tile(t + 4, a1);
        }
        __syncthreads();
    }
}

// X <- L^-T X.  The earlier rows' update of block j,
//   X[k][c] -= sum_l L[j+l][k] x_j[l][c],  k < j,
// runs on the matrix cores, 16 columns of L per tile: lane (l16, l4) holds
// L[j + 4s + l4][k0 + l16] (four consecutive words of one column) as the A
// operand and x_j[4s + l4][l16] (zero for l16 >= R) as the B operand; the
// next tile's operands are loaded while the current one is multiplied.
template <int NB, int R>
__device__ void backward_rl(const gmem<const double> L, const gmem<const double> Dinv, int Mp, double *X,
                            double *Dj, double *T) {
    static_assert(NB == 32 && R <= 16, "tiles of 16 columns, 8 MFMA steps of 4 rows");
    constexpr int S = NB / 4;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    double dn[NB * NB / 256];
    load_dinv<NB>(Dinv, Mp - NB, dn);
    for (int j = Mp - NB; j >= 0; j -= NB) {
        put_dinv<NB>(dn, Dj);
        const int nt = j / 16;  // column tiles of the earlier rows
        auto load_tile = [&](int t, double (&a)[S]) {
            const int64_t k = 16 * min(t, nt - 1) + l16;  // clamped: the loads stay unconditional
#pragma unroll
            for (int s = 0; s < S; ++s) a[s] = L[k * Mp + j + 4 * s + l4];
        };
        double a0[S], a1[S];
        if (nt > 0) load_tile(wave, a0);  // before the block solve: it does not depend on x_j
        __syncthreads();
        // x_j = Dinv_j^T b_j: x[r] = sum_{l >= r} Dinv_j[l][r] b[l]
        for (int o = tid; o < NB * R; o += 256) {
            const int r = o % NB, c = o / NB;
            double acc = 0.0;
            for (int l = r; l < NB; ++l) acc += Dj[r * (NB + 1) + l] * X[c * Mp + j + l];
            T[r * R + c] = acc;
        }
        __syncthreads();
        for (int o = tid; o < NB * R; o += 256) X[(o / NB) * Mp + j + o % NB] = T[(o % NB) * R + o / NB];
        if (j > 0) load_dinv<NB>(Dinv, j - NB, dn);
        double bx[S];
#pragma unroll
        for (int s = 0; s < S; ++s) bx[s] = l16 < R ? T[(4 * s + l4) * R + l16] : 0.0;
        auto tile = [&](int t, const double (&a)[S]) {
            dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < S; ++s) acc = mfma16x16x4(a[s], bx[s], acc);
            if (l16 < R) {
#pragma unroll
                for (int r = 0; r < 4; ++r) X[l16 * Mp + 16 * t + l4 + 4 * r] -= acc[r];
            }
        };
        for (int t = wave; t < nt; t += 8) {
            load_tile(t + 4, a1);
            tile(t, a0);
            if (t + 4 >= nt) break;
            load_tile(t + 8, a0);
            tile(t + 4, a1);
        }
        __syncthreads();
    }
}

// Apply P^-1 to up to 8 right-hand sides of one body per workgroup
// (grid.y = groups of 8 rhs).  lds: X (Mp x 8).
template <int NB>
__global__ __launch_bounds__(256) void apply_large_kernel(const PrecondApplyJob *__restrict__ jobs, int32_t n_jobs) {
    constexpr int R = 8, QP = 16;  // rhs per workgroup; partial sums per (rhs, k) of Y^T t
    extern __shared__ double lds[];
    __shared__ double Dj[NB * (NB + 1) > QP * R * 6 ? NB * (NB + 1) : QP * R * 6];
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
    double *X = lds;  // 8 columns of Mp: X[c * Mp + row]
    const bool resist = J.mode != 0;  // resistance problem: lambda = M_pp^-1 s only
    const int64_t b3 = 3 * it.w.blob0, u6 = resist ? 0 : J.nb3 + 6 * (int64_t)it.w.body;
    // with a shared reference-shape factor, the right-hand sides are taken
    // into the body frame (R^T on every 3-vector) and the results back (R)
    const gmem<const double> Rot = as_global(it.w.rot);
    if (it.w.rot) {
        for (int e = tid; e < Mp * R; e += 256) {
            const int row = e % Mp, c = e / Mp;
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
            const int row = e % Mp, c = e / Mp;
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
            const int c = tid / QP, qp = tid % QP;
            double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
            for (int l = qp; l < Mp; l += QP) {
                const double x = X[c * Mp + l];
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
                double acc = X[c * Mp + row];
#pragma unroll
                for (int k = 0; k < 6; ++k) acc += yk[k] * g[c][k];
                X[c * Mp + row] = acc;
            }
        }
        __syncthreads();
    }
    backward_rl<NB, R>(L, as_global(Dinv), Mp, X, Dj, T);
    if (it.w.rot) {
        // backward_rl ends with a barrier, so all of X is final here
        for (int e = tid; e < m * R; e += 256) {
            const int row = e % m, c = e / m;
            if (c < nr) {
                const int b = row - row % 3, k = row % 3;
                const double *xc = X + c * Mp;
                as_global(J.out)[(int64_t)(r0 + c) * J.ld + b3 + row] =
                    Rot[3 * k] * xc[b] + Rot[3 * k + 1] * xc[b + 1] + Rot[3 * k + 2] * xc[b + 2];
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
        const int row = e % m, c = e / m;
        if (c < nr) as_global(J.out)[(int64_t)(r0 + c) * J.ld + b3 + row] = X[c * Mp + row];
    }
    if (tid < R * 6 && !resist) {
        const int c = tid / 6, k = tid % 6;
        if (c < nr) as_global(J.out)[(int64_t)(r0 + c) * J.ld + u6 + k] = g[c][k];
    }
}

// ---------------------------------------------------------------------------

// Tile shapes the autotuner times: {16-row tiles per wave and pass, columns
// of L staged per chunk}; the panel is 64 columns wide in every shape and
// the stored diagonal-block inverses are 32 x 32.
struct LargeShape {
    int g, kc;
};
static constexpr LargeShape kLargeShapes[] = {{2, 32}, {2, 16}, {4, 16}, {4, 8}};  // the first: small batches
constexpr int kLargeVariants = (int)(sizeof(kLargeShapes) / sizeof(kLargeShapes[0]));

int large_variant_count() { return kLargeVariants; }
void large_variant_shape(int variant, int *nb, int *row_tiles, int *chunk) {
    *nb = kPanel;
    *row_tiles = kLargeShapes[variant].g;
    *chunk = kLargeShapes[variant].kc;
}

template <int V>
static void launch_chol(const BigBody *items, int32_t n_items, hipStream_t s) {
    constexpr LargeShape sh = kLargeShapes[V];
    hipLaunchKernelGGL((chol_panel_kernel<sh.g, sh.kc>), dim3(n_items), dim3(256), 0, s, items);
}

hipError_t launch_precond_build_large(const BigBody *items, int32_t n_items, int max_Mp, int variant, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (variant < 0 || variant >= kLargeVariants) return hipErrorInvalidValue;
    hipLaunchKernelGGL(assemble_large_kernel, dim3(n_items, asm_tiles(max_Mp)), dim3(256), 0, s, items);
    switch (variant) {
        case 0: launch_chol<0>(items, n_items, s); break;
        case 1: launch_chol<1>(items, n_items, s); break;
        case 2: launch_chol<2>(items, n_items, s); break;
        default: launch_chol<3>(items, n_items, s); break;
    }
    static_assert(kLargeVariants == 4, "launch switch covers every shape");
    return hipGetLastError();
}

hipError_t launch_precond_apply_large(const PrecondApplyJob *jobs, int32_t n_jobs, int64_t n_wg, int32_t max_rhs,
                                      int max_Mp, hipStream_t s) {
    if (n_wg <= 0 || max_rhs <= 0) return hipSuccess;
    const size_t lds = (size_t)max_Mp * 8 * sizeof(double);
    dim3 g((unsigned)n_wg, (max_rhs + 7) / 8);
    hipLaunchKernelGGL(apply_large_kernel<32>, g, dim3(256), lds, s, jobs, n_jobs);
    return hipGetLastError();
}

}  // namespace rmb

// Krylov vector kernels for GMRES (Sec. 2.2.2): classical Gram-Schmidt with
// one re-orthogonalisation (CGS2), norms, basis combinations and updates.
//
// Every launch may cover several independent systems.  A system owns the
// workgroups [wg_begin, wg_begin + n_seg) of the launch; workgroup s of a
// system covers elements [s*L, (s+1)*L) of its vectors, L = n_chunk * 512
// (n_chunk keeps n_seg <= kMaxSeg).  Dot products are reduced in two
// stages: each workgroup writes its partials, and every workgroup of the
// next launch sums all of a system's partials itself, in one fixed order.
// All workgroups therefore hold bitwise the same coefficients, independent
// of scheduling and of what else shares the launch, and no workgroup ever
// waits on another inside a launch (no device-wide fences or atomics).
#include "rmb_body.h"

namespace rmb {

constexpr int kThreads = 256;
constexpr int kPer = kSeg / kThreads;  // elements per thread and chunk
constexpr int kMaxKK = 256;            // largest basis handled (restart <= 255)

__device__ __forceinline__ int find_wg_job(const KrylovJob *__restrict__ jobs, int32_t n_jobs, int64_t w) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// This workgroup's element range [b0, b1) of its system.
struct Range {
    int64_t b0, b1;
};
__device__ __forceinline__ Range seg_range(const KrylovJob &J, int sg) {
    const int64_t len = (int64_t)J.n_chunk * kSeg;
    const int64_t b0 = (int64_t)sg * len;
    return Range{b0, min(J.n, b0 + len)};
}

// One DPP step on a double: x + (x moved by CTRL); lanes outside ROW_MASK or
// shifted in from outside a row read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add_d(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return x + __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Total over the 64 lanes of a wave (row shifts leave each row's sum in its
// lane 15, row broadcasts carry them to lane 63), returned to every lane.
__device__ __forceinline__ double wave_total(double v) {
    v = dpp_add_d<0x111, 0xf>(v);
    v = dpp_add_d<0x112, 0xf>(v);
    v = dpp_add_d<0x114, 0xf>(v);
    v = dpp_add_d<0x118, 0xf>(v);
    v = dpp_add_d<0x142, 0xa>(v);
    v = dpp_add_d<0x143, 0xc>(v);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Block-wide sums of per-thread values: each wave totals its lanes and lane
// 0 stores red[k][wave]; after a sync, block_sum(red, k) adds the 4 wave
// results in order.
__device__ __forceinline__ void stash_wave_sum(double v, int k, double *red) {
    v = wave_total(v);
    if ((threadIdx.x & 63) == 0) red[k * 4 + (threadIdx.x >> 6)] = v;
}
__device__ __forceinline__ double block_sum(const double *red, int k) {
    return ((red[4 * k] + red[4 * k + 1]) + red[4 * k + 2]) + red[4 * k + 3];
}

// out[k] = sum_{s < n_seg} P[k*n_seg + s] for k < kk, in a fixed order:
// Q threads per k take strided partial sums (s = q, q+Q, ..., eight loads in
// flight), then a fixed tree over q.  Ends with a sync.
__device__ __forceinline__ void reduce_partials(const double *__restrict__ P, int kk, int n_seg, double *out, double *red) {
    int Q = kThreads;
    while (Q > 1 && Q * kk > kThreads) Q >>= 1;
    const int t = threadIdx.x;
    for (int k0 = 0; k0 < kk; k0 += kThreads / Q) {
        const int k = k0 + t / Q, q = t % Q;
        double acc = 0.0;
        if (k < kk) {
            const gmem<const double> Pk = as_global(P + (int64_t)k * n_seg);
            int sg = q;
            for (; sg + 7 * Q < n_seg; sg += 8 * Q) {
                double v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = Pk[sg + i * Q];
#pragma unroll
                for (int i = 0; i < 8; ++i) acc += v[i];
            }
            for (; sg < n_seg; sg += Q) acc += Pk[sg];
        }
        red[t] = acc;
        __syncthreads();
        for (int w = Q / 2; w >= 1; w >>= 1) {
            if (q < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (q == 0 && k < kk) out[k] = red[t];
        __syncthreads();
    }
}

// Partial dot products <V_k, w> over [r.b0, r.b1) for k < kk into red (see
// stash_wave_sum), eight basis vectors at a time so that their loads are in
// flight together and their wave reductions interleave.
__device__ __forceinline__ void block_dots(const KrylovJob &J, Range r, int kk, double *red) {
    constexpr int C = 8;
    int k = 0;
    for (; k < kk; k += C) {
        const int nc = min(C, kk - k);
        double acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0.0;
        for (int64_t e0 = r.b0 + threadIdx.x; e0 < r.b1; e0 += kSeg) {
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int64_t e = e0 + u * kThreads;
                if (e >= r.b1) continue;
                const double we = as_global(J.w)[e];
                if (nc == C) {
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[c] += as_global(J.V)[(k + c) * J.ldv + e] * we;
                } else {
                    for (int c = 0; c < nc; ++c) acc[c] += as_global(J.V)[(k + c) * J.ldv + e] * we;
                }
            }
        }
        if (nc == C) {
#pragma unroll
            for (int c = 0; c < C; ++c) stash_wave_sum(acc[c], k + c, red);
        } else {
            for (int c = 0; c < nc; ++c) stash_wave_sum(acc[c], k + c, red);
        }
    }
}

// w -= sum_k h[k] V_k over [r.b0, r.b1), subtracting in the order k = 0, 1,
// ...  (eight basis vectors loaded at a time), and returns this thread's part
// of ||w||^2 after the update.
__device__ __forceinline__ double block_subtract(const KrylovJob &J, Range r, const double *h, int kk) {
    constexpr int C = 8;
    double sq = 0.0;
    for (int64_t e0 = r.b0 + threadIdx.x; e0 < r.b1; e0 += kSeg) {
        double wv[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t e = e0 + u * kThreads;
            wv[u] = e < r.b1 ? as_global(J.w)[e] : 0.0;
        }
        int k = 0;
        for (; k + C <= kk; k += C) {
            double v[C][kPer];
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int u = 0; u < kPer; ++u) {
                    const int64_t e = e0 + u * kThreads;
                    v[c][u] = e < r.b1 ? as_global(J.V)[(k + c) * J.ldv + e] : 0.0;
                }
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int u = 0; u < kPer; ++u) wv[u] -= h[k + c] * v[c][u];
        }
        for (; k < kk; ++k) {
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int64_t e = e0 + u * kThreads;
                if (e < r.b1) wv[u] -= h[k] * as_global(J.V)[k * J.ldv + e];
            }
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t e = e0 + u * kThreads;
            if (e < r.b1) {
                if (kk > 0) as_global(J.w)[e] = wv[u];
                sq += wv[u] * wv[u];
            }
        }
    }
    return sq;
}

// pass 1: partials P1 of <V_k, w>
__global__ __launch_bounds__(kThreads) void orth_dots_kernel(const KrylovJob *__restrict__ jobs, int32_t n_jobs) {
    __shared__ double red[kMaxKK * 4];
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int kk = J.kk;
    if (kk == 0) return;
    block_dots(J, seg_range(J, sg), kk, red);
    __syncthreads();
    for (int k = threadIdx.x; k < kk; k += kThreads) as_global(J.P1)[(int64_t)k * J.n_seg + sg] = block_sum(red, k);
}

// pass 2: h1 = sum of P1; w -= V h1; partials P2 of <V_k, w>.  Workgroup 0
// keeps h1 in hred.
__global__ __launch_bounds__(kThreads) void orth_update_dots_kernel(const KrylovJob *__restrict__ jobs,
                                                                    int32_t n_jobs) {
    __shared__ double red[kMaxKK * 4];
    __shared__ double h[kMaxKK];
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int kk = J.kk;
    if (kk == 0) return;
    reduce_partials(J.P1, kk, J.n_seg, h, red);
    if (sg == 0)
        for (int k = threadIdx.x; k < kk; k += kThreads) as_global(J.hred)[k] = h[k];
    const Range r = seg_range(J, sg);
    (void)block_subtract(J, r, h, kk);
    block_dots(J, r, kk, red);
    __syncthreads();
    for (int k = threadIdx.x; k < kk; k += kThreads) as_global(J.P2)[(int64_t)k * J.n_seg + sg] = block_sum(red, k);
}

// pass 3: h2 = sum of P2; w -= V h2; partials P3 of ||w||^2.  Workgroup 0
// writes hcol[k] = h1 + h2.
__global__ __launch_bounds__(kThreads) void orth_update_norm_kernel(const KrylovJob *__restrict__ jobs,
                                                                    int32_t n_jobs) {
    __shared__ double red[kThreads];
    __shared__ double h[kMaxKK];
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int kk = J.kk;
    if (kk > 0) {
        reduce_partials(J.P2, kk, J.n_seg, h, red);
        if (sg == 0)
            for (int k = threadIdx.x; k < kk; k += kThreads) as_global(J.hcol)[k] = as_global(J.hred)[k] + h[k];
    }
    const double sq = block_subtract(J, seg_range(J, sg), h, kk);
    stash_wave_sum(sq, 0, red);
    __syncthreads();
    if (threadIdx.x == 0) as_global(J.P3)[sg] = block_sum(red, 0);
}

// pass 4: beta = sqrt(sum of P3); vnext = w / beta.  Workgroup 0 writes
// hcol[kk] = beta.
__global__ __launch_bounds__(kThreads) void orth_normalise_kernel(const KrylovJob *__restrict__ jobs,
                                                                  int32_t n_jobs) {
    __shared__ double red[kThreads];
    __shared__ double nrm[1];
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    reduce_partials(J.P3, 1, J.n_seg, nrm, red);
    const double beta = sqrt(nrm[0]);
    if (sg == 0 && threadIdx.x == 0) as_global(J.hcol)[J.kk] = beta;
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    const Range r = seg_range(J, sg);
    for (int64_t e = r.b0 + threadIdx.x; e < r.b1; e += kThreads) as_global(J.vnext)[e] = as_global(J.w)[e] * inv;
}

hipError_t launch_orthogonalise(const KrylovJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    dim3 g((unsigned)n_wg), b(kThreads);
    hipLaunchKernelGGL(orth_dots_kernel, g, b, 0, s, jobs, n_jobs);
    hipLaunchKernelGGL(orth_update_dots_kernel, g, b, 0, s, jobs, n_jobs);
    hipLaunchKernelGGL(orth_update_norm_kernel, g, b, 0, s, jobs, n_jobs);
    hipLaunchKernelGGL(orth_normalise_kernel, g, b, 0, s, jobs, n_jobs);
    return hipGetLastError();
}

// w = sum_{k < kk} coef[k] V_k
__global__ __launch_bounds__(kThreads) void combine_kernel(const KrylovJob *__restrict__ jobs, int32_t n_jobs) {
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const Range r = seg_range(J, (int)(wgi - J.wg_begin));
    for (int64_t e = r.b0 + threadIdx.x; e < r.b1; e += kThreads) {
        double acc = 0.0;
        for (int k = 0; k < J.kk; ++k) acc += as_global(J.coef)[k] * as_global(J.V)[k * J.ldv + e];
        as_global(J.w)[e] = acc;
    }
}

hipError_t launch_combine(const KrylovJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)n_wg), dim3(kThreads), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

// x += t
__global__ __launch_bounds__(kThreads) void axpy_kernel(const KrylovJob *__restrict__ jobs, int32_t n_jobs) {
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const Range r = seg_range(J, (int)(wgi - J.wg_begin));
    for (int64_t e = r.b0 + threadIdx.x; e < r.b1; e += kThreads) as_global(J.x)[e] += as_global(J.t)[e];
}

hipError_t launch_axpy(const KrylovJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)n_wg), dim3(kThreads), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

// Squared norms of the body part of the last correction (t) and of the
// updated iterate (x), for the velocity-error estimate of a solve: one
// workgroup per job, each thread summing a strided range, then the
// workgroup's fixed-order reduction.
__global__ __launch_bounds__(kThreads) void unorm_kernel(const KrylovJob *__restrict__ jobs, int32_t n_jobs) {
    __shared__ double red[kThreads];
    const KrylovJob &J = jobs[blockIdx.x];
    double st = 0.0, sx = 0.0;
    for (int64_t e = J.u0 + threadIdx.x; e < J.n; e += kThreads) {
        const double t = as_global(J.t)[e], x = as_global(J.x)[e];
        st = fma(t, t, st);
        sx = fma(x, x, sx);
    }
    stash_wave_sum(st, 0, red);
    __syncthreads();
    const double tt = block_sum(red, 0);
    __syncthreads();
    stash_wave_sum(sx, 0, red);
    __syncthreads();
    const double xx = block_sum(red, 0);
    if (threadIdx.x == 0) {
        as_global(J.hcol)[1] = tt;
        as_global(J.hcol)[2] = xx;
    }
}

hipError_t launch_unorm(const KrylovJob *jobs, int32_t n_jobs, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(unorm_kernel, dim3((unsigned)n_jobs), dim3(kThreads), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

__global__ void build_rhs_kernel(const double *__restrict__ FT, const double *__restrict__ slip, int64_t nb3,
                                 int64_t n, double *__restrict__ b) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    b[e] = e < nb3 ? (slip ? slip[e] : 0.0) : -FT[e - nb3];
}

hipError_t launch_build_rhs(const double *FT, const double *slip, int64_t nb, int64_t N, double *b,
                            hipStream_t s) {
    const int64_t n = 3 * nb + 6 * N;
    hipLaunchKernelGGL(build_rhs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, FT, slip, 3 * nb,
                       n, b);
    return hipGetLastError();
}

__global__ void blob_body_kernel(const int64_t *__restrict__ off, int64_t N, int32_t *__restrict__ bb) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    for (int64_t i = off[p]; i < off[p + 1]; ++i) bb[i] = (int32_t)p;
}

hipError_t launch_blob_body(const int64_t *off, int64_t N, int32_t *blob_body, hipStream_t s) {
    hipLaunchKernelGGL(blob_body_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, off, N, blob_body);
    return hipGetLastError();
}

}  // namespace rmb

// Krylov vector kernels for GMRES (Sec. 2.2.2): classical Gram-Schmidt with
// one re-orthogonalisation (CGS2), norms, basis combinations and updates.
//
// Every launch may cover several independent systems.  A system owns the
// workgroups [wg_begin, wg_begin + n_seg) of the launch; workgroup s of a
// system covers elements [s*2048, (s+1)*2048) of its vectors.  Dot products
// are reduced in two stages with a fixed order (per-workgroup partials, then
// a sequential sum over workgroups done identically by every consumer
// workgroup), so results are bitwise reproducible and independent of what
// else shares the launch.
#include "rmb_body.h"

namespace rmb {

constexpr int kThreads = 256;
constexpr int kPer = kSeg / kThreads;  // 8 elements per thread
constexpr int kMaxKK = 256;            // largest basis handled (restart <= 255)

__device__ __forceinline__ int find_wg_job(const KrylovJob *__restrict__ jobs, int32_t n_jobs, int64_t w) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum of per-thread values for kk vectors at once: each wave
// reduces with cross-lane shuffles, lane 0 stores to red[k][wave]; the caller
// syncs and sums the 4 wave results in order.
__device__ __forceinline__ void stash_wave_sum(double v, int k, double *red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[k * 4 + (threadIdx.x >> 6)] = v;
}

// h[k] = sum over segments of P[k][seg], k < kk, into shared memory.
__device__ __forceinline__ void reduce_partials_to_shared(const double *__restrict__ P, int n_seg, int kk,
                                                          double *sh) {
    for (int k = threadIdx.x; k < kk; k += blockDim.x) {
        double acc = 0.0;
        for (int sgi = 0; sgi < n_seg; ++sgi) acc += P[(int64_t)k * n_seg + sgi];
        sh[k] = acc;
    }
}

// pass 1: P1[k][seg] = <V_k, w>_seg
__global__ __launch_bounds__(kThreads) void orth_dots_kernel(const KrylovJob *__restrict__ jobs, int32_t n_jobs) {
    __shared__ double red[kMaxKK * 4];
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int kk = J.kk;
    if (kk == 0) return;
    const int64_t e0 = (int64_t)sg * kSeg + threadIdx.x;
    double wv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t e = e0 + u * kThreads;
        wv[u] = e < J.n ? J.w[e] : 0.0;
    }
    for (int k = 0; k < kk; ++k) {
        const double *Vk = J.V + k * J.ldv;
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t e = e0 + u * kThreads;
            if (e < J.n) acc += Vk[e] * wv[u];
        }
        stash_wave_sum(acc, k, red);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kk; k += kThreads)
        J.P1[(int64_t)k * J.n_seg + sg] = ((red[4 * k] + red[4 * k + 1]) + red[4 * k + 2]) + red[4 * k + 3];
}

// pass 2: w -= V h1 (h1 from P1), then P2[k][seg] = <V_k, w>_seg
__global__ __launch_bounds__(kThreads) void orth_update_dots_kernel(const KrylovJob *__restrict__ jobs,
                                                                    int32_t n_jobs) {
    __shared__ double red[kMaxKK * 4];
    __shared__ double h[kMaxKK];
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int kk = J.kk;
    if (kk == 0) return;
    reduce_partials_to_shared(J.P1, J.n_seg, kk, h);
    __syncthreads();
    const int64_t e0 = (int64_t)sg * kSeg + threadIdx.x;
    double wv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t e = e0 + u * kThreads;
        wv[u] = e < J.n ? J.w[e] : 0.0;
    }
    for (int k = 0; k < kk; ++k) {
        const double *Vk = J.V + k * J.ldv;
        const double hk = h[k];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t e = e0 + u * kThreads;
            if (e < J.n) wv[u] -= hk * Vk[e];
        }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t e = e0 + u * kThreads;
        if (e < J.n) J.w[e] = wv[u];
    }
    for (int k = 0; k < kk; ++k) {
        const double *Vk = J.V + k * J.ldv;
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t e = e0 + u * kThreads;
            if (e < J.n) acc += Vk[e] * wv[u];
        }
        stash_wave_sum(acc, k, red);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kk; k += kThreads)
        J.P2[(int64_t)k * J.n_seg + sg] = ((red[4 * k] + red[4 * k + 1]) + red[4 * k + 2]) + red[4 * k + 3];
}

// pass 3: w -= V h2 (h2 from P2); P3[seg] = ||w||^2_seg; hcol[k] = h1 + h2
__global__ __launch_bounds__(kThreads) void orth_update_norm_kernel(const KrylovJob *__restrict__ jobs,
                                                                    int32_t n_jobs) {
    __shared__ double red[4];
    __shared__ double h[kMaxKK];
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int kk = J.kk;
    const int64_t e0 = (int64_t)sg * kSeg + threadIdx.x;
    double wv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t e = e0 + u * kThreads;
        wv[u] = e < J.n ? J.w[e] : 0.0;
    }
    if (kk > 0) {
        reduce_partials_to_shared(J.P2, J.n_seg, kk, h);
        __syncthreads();
        for (int k = 0; k < kk; ++k) {
            const double *Vk = J.V + k * J.ldv;
            const double hk = h[k];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int64_t e = e0 + u * kThreads;
                if (e < J.n) wv[u] -= hk * Vk[e];
            }
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t e = e0 + u * kThreads;
            if (e < J.n) J.w[e] = wv[u];
        }
        if (sg == 0) {
            // hcol[k] = h1[k] + h2[k]
            for (int k = threadIdx.x; k < kk; k += kThreads) {
                double a1 = 0.0;
                for (int s = 0; s < J.n_seg; ++s) a1 += J.P1[(int64_t)k * J.n_seg + s];
                J.hcol[k] = a1 + h[k];
            }
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) acc += wv[u] * wv[u];
    stash_wave_sum(acc, 0, red);
    __syncthreads();
    if (threadIdx.x == 0) J.P3[sg] = ((red[0] + red[1]) + red[2]) + red[3];
}

// pass 4: beta = sqrt(sum P3); vnext = w / beta; hcol[kk] = beta
__global__ __launch_bounds__(kThreads) void orth_normalise_kernel(const KrylovJob *__restrict__ jobs,
                                                                  int32_t n_jobs) {
    __shared__ double beta_s;
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int s = 0; s < J.n_seg; ++s) acc += J.P3[s];
        beta_s = sqrt(acc);
        if (sg == 0) J.hcol[J.kk] = beta_s;
    }
    __syncthreads();
    const double beta = beta_s;
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    const int64_t e0 = (int64_t)sg * kSeg + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t e = e0 + u * kThreads;
        if (e < J.n) J.vnext[e] = J.w[e] * inv;
    }
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

// norm only: P3 then hcol[0] = ||w||
__global__ __launch_bounds__(kThreads) void norm_final_kernel(const KrylovJob *__restrict__ jobs, int32_t n_jobs) {
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    if (sg == 0 && threadIdx.x == 0) {
        double acc = 0.0;
        for (int s = 0; s < J.n_seg; ++s) acc += J.P3[s];
        J.hcol[0] = sqrt(acc);
    }
}

__global__ __launch_bounds__(kThreads) void norm_partial_kernel(const KrylovJob *__restrict__ jobs, int32_t n_jobs) {
    __shared__ double red[4];
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int64_t e0 = (int64_t)sg * kSeg + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t e = e0 + u * kThreads;
        if (e < J.n) acc += J.w[e] * J.w[e];
    }
    stash_wave_sum(acc, 0, red);
    __syncthreads();
    if (threadIdx.x == 0) J.P3[sg] = ((red[0] + red[1]) + red[2]) + red[3];
}

hipError_t launch_norm(const KrylovJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(norm_partial_kernel, dim3((unsigned)n_wg), dim3(kThreads), 0, s, jobs, n_jobs);
    hipLaunchKernelGGL(norm_final_kernel, dim3((unsigned)n_wg), dim3(kThreads), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

// w = sum_{k < kk} coef[k] V_k
__global__ __launch_bounds__(kThreads) void combine_kernel(const KrylovJob *__restrict__ jobs, int32_t n_jobs) {
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int64_t e0 = (int64_t)sg * kSeg + threadIdx.x;
    double acc[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) acc[u] = 0.0;
    for (int k = 0; k < J.kk; ++k) {
        const double c = J.coef[k];
        const double *Vk = J.V + k * J.ldv;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t e = e0 + u * kThreads;
            if (e < J.n) acc[u] += c * Vk[e];
        }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t e = e0 + u * kThreads;
        if (e < J.n) J.w[e] = acc[u];
    }
}

hipError_t launch_combine(const KrylovJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)n_wg), dim3(kThreads), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void axpy_kernel(const KrylovJob *__restrict__ jobs, int32_t n_jobs) {
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int64_t e0 = (int64_t)sg * kSeg + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t e = e0 + u * kThreads;
        if (e < J.n) J.x[e] += J.t[e];
    }
}

hipError_t launch_axpy(const KrylovJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)n_wg), dim3(kThreads), 0, s, jobs, n_jobs);
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

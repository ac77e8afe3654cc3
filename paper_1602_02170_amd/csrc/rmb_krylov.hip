// Krylov vector kernels for GMRES (Sec. 2.2.2): classical Gram-Schmidt with
// one re-orthogonalisation (CGS2), norms, basis combinations and updates.
//
// Every launch may cover several independent systems.  A system owns the
// workgroups [wg_begin, wg_begin + n_seg) of the launch; workgroup s of a
// system covers elements [s*512, (s+1)*512) of its vectors.  Dot products
// are reduced in two stages: per-workgroup partials, then a fixed-order sum
// done by whichever workgroup of the system finishes last.  The order depends
// only on the system's own sizes, so results are bitwise reproducible and
// independent of what else shares the launch.
#include "rmb_body.h"

namespace rmb {

constexpr int kThreads = 256;
constexpr int kPer = kSeg / kThreads;  // elements per thread
constexpr int kMaxKK = 256;            // largest basis handled (restart <= 255)

__device__ __forceinline__ int find_wg_job(const KrylovJob *__restrict__ jobs, int32_t n_jobs, int64_t w) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
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
// 0 stores red[k][wave]; the caller syncs and adds the 4 wave results in
// order.
__device__ __forceinline__ void stash_wave_sum(double v, int k, double *red) {
    v = wave_total(v);
    if ((threadIdx.x & 63) == 0) red[k * 4 + (threadIdx.x >> 6)] = v;
}

// Partial dot products <V_k, w> of this workgroup's elements for k < kk,
// four basis vectors at a time so that their reductions interleave.
__device__ __forceinline__ void block_dots(const KrylovJob &J, const double *wv, int64_t e0, int kk, double *red) {
    int k = 0;
    for (; k + 4 <= kk; k += 4) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double *Vk = J.V + (k + c) * J.ldv;
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int64_t e = e0 + u * 256;
                if (e < J.n) acc[c] += Vk[e] * wv[u];
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) stash_wave_sum(acc[c], k + c, red);
    }
    for (; k < kk; ++k) {
        const double *Vk = J.V + k * J.ldv;
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t e = e0 + u * 256;
            if (e < J.n) acc += Vk[e] * wv[u];
        }
        stash_wave_sum(acc, k, red);
    }
}

// Writes this workgroup's partials, then lets the last workgroup of the
// system to finish (atomic ticket) reduce them: out[k] = sum_s P[k][s] for
// k < kk, in a fixed order (strided partial sums per thread, then a fixed
// tree), so the result does not depend on which workgroup finishes last.
// Returns true in the reducing workgroup.
__device__ bool last_block_reduce(const KrylovJob &J, const double *P, int kk, double *out, double *red) {
    __shared__ bool last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(J.counter, 1u) == (unsigned)(J.n_seg - 1);
    __syncthreads();
    if (!last) return false;
    __threadfence();
    int Q = kThreads;
    while (Q > 1 && Q * kk > kThreads) Q >>= 1;
    const int t = threadIdx.x;
    for (int k0 = 0; k0 < kk; k0 += kThreads / Q) {
        const int k = k0 + t / Q, q = t % Q;
        double acc = 0.0;
        if (k < kk)
            for (int sg = q; sg < J.n_seg; sg += Q) acc += __builtin_nontemporal_load(&P[(int64_t)k * J.n_seg + sg]);
        red[t] = acc;
        __syncthreads();
        for (int w = Q / 2; w >= 1; w >>= 1) {
            if (q < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (q == 0 && k < kk) out[k] = red[t];
        __syncthreads();
    }
    if (threadIdx.x == 0) *J.counter = 0u;
    return true;
}

// pass 1: partial <V_k, w>; the last workgroup forms h1
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
    block_dots(J, wv, e0, kk, red);
    __syncthreads();
    for (int k = threadIdx.x; k < kk; k += kThreads)
        J.P1[(int64_t)k * J.n_seg + sg] = ((red[4 * k] + red[4 * k + 1]) + red[4 * k + 2]) + red[4 * k + 3];
    last_block_reduce(J, J.P1, kk, J.hred, red);
}

// pass 2: w -= V h1, partial <V_k, w>; the last workgroup forms h2 and
// hcol[k] = h1 + h2
__global__ __launch_bounds__(kThreads) void orth_update_dots_kernel(const KrylovJob *__restrict__ jobs,
                                                                    int32_t n_jobs) {
    __shared__ double red[kMaxKK * 4];
    __shared__ double h[kMaxKK];
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const int kk = J.kk;
    if (kk == 0) return;
    for (int k = threadIdx.x; k < kk; k += kThreads) h[k] = J.hred[k];
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
    block_dots(J, wv, e0, kk, red);
    __syncthreads();
    for (int k = threadIdx.x; k < kk; k += kThreads)
        J.P2[(int64_t)k * J.n_seg + sg] = ((red[4 * k] + red[4 * k + 1]) + red[4 * k + 2]) + red[4 * k + 3];
    if (last_block_reduce(J, J.P2, kk, J.hred + kMaxKK, red)) {
        for (int k = threadIdx.x; k < kk; k += kThreads) J.hcol[k] = h[k] + J.hred[kMaxKK + k];
    }
}

// pass 3: w -= V h2, partial ||w||^2; the last workgroup forms the norm
__global__ __launch_bounds__(kThreads) void orth_update_norm_kernel(const KrylovJob *__restrict__ jobs,
                                                                    int32_t n_jobs) {
    __shared__ double red[kThreads];
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
        for (int k = threadIdx.x; k < kk; k += kThreads) h[k] = J.hred[kMaxKK + k];
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
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) acc += wv[u] * wv[u];
    stash_wave_sum(acc, 0, red);
    __syncthreads();
    if (threadIdx.x == 0) J.P3[sg] = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    if (last_block_reduce(J, J.P3, 1, J.hred + 2 * kMaxKK, red)) {
        if (threadIdx.x == 0) {
            const double beta = sqrt(J.hred[2 * kMaxKK]);
            J.hred[2 * kMaxKK] = beta;
            J.hcol[kk] = beta;
        }
    }
}

// pass 4: vnext = w / beta
__global__ __launch_bounds__(kThreads) void orth_normalise_kernel(const KrylovJob *__restrict__ jobs,
                                                                  int32_t n_jobs) {
    const int64_t wgi = blockIdx.x;
    const KrylovJob &J = jobs[find_wg_job(jobs, n_jobs, wgi)];
    const int sg = (int)(wgi - J.wg_begin);
    const double beta = J.hred[2 * kMaxKK];
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

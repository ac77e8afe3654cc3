// Context management, validation and the blob mobility product entry points.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "rmb_ctx.h"

// Workspace of rmb_mobility_matvec_noalloc: a static device array, so that
// the entry point allocates nothing.  Every device the library runs on holds
// its own copy until the process ends.  Host code never uses the array's
// name for memory: its device address comes from hipGetSymbolAddress, per
// device, when a context is created on that device.
constexpr size_t kNoAllocBytes = size_t(128) << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace rmb {

rmb_status fail(rmb_ctx ctx, rmb_status st, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

rmb_status enter(rmb_ctx ctx, hipStream_t s) {
    RMB_HIP(ctx, hipSetDevice(ctx->device));
    if (ctx->any_stream && ctx->last_stream != s) RMB_HIP(ctx, hipStreamSynchronize(ctx->last_stream));
    ctx->last_stream = s;
    ctx->any_stream = true;
    ctx->err.clear();
    return RMB_OK;
}

rmb_status ctx_scratch(rmb_ctx ctx, size_t bytes, void **out) {
    if (bytes <= ctx->scratch_bytes) {
        *out = ctx->scratch;
        return RMB_OK;
    }
    // the old scratch may still be read by queued work on the current stream
    if (ctx->scratch) {
        RMB_HIP(ctx, hipStreamSynchronize(ctx->last_stream));
        ctx->arena->free(ctx->scratch);
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    void *p = ctx->arena->alloc(want);
    if (!p) {
        want = bytes;
        p = ctx->arena->alloc(want);
    }
    if (!p)
        return fail(ctx, RMB_ENOMEM, "scratch of %zu bytes exceeds the device-memory budget (%zu in use of %zu)",
                    bytes, ctx->arena->in_use(), ctx->arena->budget());
    ctx->scratch = p;
    ctx->scratch_bytes = want;
    *out = p;
    return RMB_OK;
}

rmb_status pinned(rmb_ctx ctx, size_t bytes, void **out) {
    if (bytes > ctx->pinned_bytes) {
        if (ctx->pinned) {
            RMB_HIP(ctx, hipStreamSynchronize(ctx->last_stream));
            RMB_HIP(ctx, hipHostFree(ctx->pinned));
            ctx->pinned = nullptr;
            ctx->pinned_bytes = 0;
        }
        size_t want = std::max<size_t>(bytes, 1 << 16);
        RMB_HIP(ctx, hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
        ctx->pinned_bytes = want;
    }
    *out = ctx->pinned;
    return RMB_OK;
}

void *pinned_lease(rmb_ctx ctx, size_t bytes, size_t *got) {
    auto &c = ctx->pinned_cache;
    size_t best = c.size();
    for (size_t i = 0; i < c.size(); ++i)
        if (c[i].second >= bytes && (best == c.size() || c[i].second < c[best].second)) best = i;
    if (best < c.size()) {
        void *p = c[best].first;
        *got = c[best].second;
        c.erase(c.begin() + best);
        return p;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    *got = bytes;
    return p;
}

void pinned_give(rmb_ctx ctx, void *p, size_t bytes) {
    if (!p) return;
    auto &c = ctx->pinned_cache;
    c.emplace_back(p, bytes);
    if (c.size() > 8) {  // keep the largest few
        size_t small = 0;
        for (size_t i = 1; i < c.size(); ++i)
            if (c[i].second < c[small].second) small = i;
        (void)hipHostFree(c[small].first);
        c.erase(c.begin() + small);
    }
}

rmb_status check_system(rmb_ctx ctx, const rmb_system *sys, bool need_bodies) {
    if (!sys) return fail(ctx, RMB_EINVAL, "system is NULL");
    if (sys->n_blobs < 1) return fail(ctx, RMB_EINVAL, "n_blobs must be >= 1 (got %lld)", (long long)sys->n_blobs);
    if (sys->n_blobs > (int64_t(1) << 31) / 3)
        return fail(ctx, RMB_EINVAL, "n_blobs %lld is above the supported maximum", (long long)sys->n_blobs);
    if (!sys->pos) return fail(ctx, RMB_EINVAL, "pos is NULL");
    if (!(sys->a > 0.0) || !std::isfinite(sys->a)) return fail(ctx, RMB_EINVAL, "blob radius a must be > 0");
    if (!(sys->eta > 0.0) || !std::isfinite(sys->eta)) return fail(ctx, RMB_EINVAL, "viscosity eta must be > 0");
    if (sys->geometry != RMB_GEOM_FREE && sys->geometry != RMB_GEOM_WALL)
        return fail(ctx, RMB_EINVAL, "unknown geometry %d", sys->geometry);
    if (need_bodies) {
        if (sys->n_bodies < 1) return fail(ctx, RMB_EINVAL, "n_bodies must be >= 1");
        if (!sys->body_off || !sys->q) return fail(ctx, RMB_EINVAL, "body_off and q are required");
        if (sys->body_off[0] != 0) return fail(ctx, RMB_EINVAL, "body_off[0] must be 0");
        for (int64_t p = 0; p < sys->n_bodies; ++p)
            if (sys->body_off[p + 1] <= sys->body_off[p])
                return fail(ctx, RMB_EINVAL, "body_off must be strictly increasing (body %lld)", (long long)p);
        if (sys->body_off[sys->n_bodies] != sys->n_blobs)
            return fail(ctx, RMB_EINVAL, "body_off[n_bodies] must equal n_blobs");
    }
    return RMB_OK;
}

rmb_status check_positions(rmb_ctx ctx, const rmb_system *sys, int *flag_dev, hipStream_t s) {
    int *h = nullptr;
    RMB_TRY(pinned(ctx, sizeof(int), (void **)&h));
    RMB_HIP(ctx, hipMemsetAsync(flag_dev, 0, sizeof(int), s));
    RMB_HIP(ctx, launch_validate_positions(sys->pos, sys->n_blobs, sys->geometry == RMB_GEOM_WALL, sys->blob_shift,
                                           flag_dev, s));
    RMB_HIP(ctx, hipMemcpyAsync(h, flag_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    RMB_HIP(ctx, hipStreamSynchronize(s));
    if (*h & 1) return fail(ctx, RMB_EINVAL, "non-finite blob position");
    if (*h & 2) return fail(ctx, RMB_EINVAL, "a blob has z <= 0 in wall geometry");
    if (*h & 32) return fail(ctx, RMB_EINVAL, "blob_shift must be finite and >= 0");
    return RMB_OK;
}

static hipEvent_t take_event(rmb_ctx ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    // timestamps only: no system-scope fence when the marker completes (the
    // fence costs microseconds of idle time around every timed launch)
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

rmb_status pair_launch(rmb_ctx ctx, int precision, bool wall, const PairJob *jobs, int32_t n_jobs, int64_t n_tiles,
                       hipStream_t s) {
    const int kid = (precision == RMB_PREC_FP32_PAIRS ? 0 : 2) + (wall ? 0 : 1);
    hipEvent_t a = nullptr, b = nullptr;
    if (ctx->timing) {
        a = take_event(ctx);
        b = take_event(ctx);
        if (!a || !b) {
            if (a) ctx->event_pool.push_back(a);
            if (b) ctx->event_pool.push_back(b);
            a = b = nullptr;
        }
        if (a) RMB_HIP(ctx, hipEventRecord(a, s));
    }
    RMB_HIP(ctx, launch_pair_tiles(precision, wall, jobs, n_jobs, n_tiles, s));
    if (a) {
        RMB_HIP(ctx, hipEventRecord(b, s));
        ctx->pending.push_back({kid, a, b});
    }
    return RMB_OK;
}

rmb_status sym_launch(rmb_ctx ctx, int precision, bool wall, int B, const SymJob *jobs, int32_t n_jobs,
                      int64_t n_tiles, hipStream_t s) {
    const int kid = (precision == RMB_PREC_FP32_PAIRS ? 0 : 2) + (wall ? 0 : 1);
    hipEvent_t a = nullptr, b = nullptr;
    if (ctx->timing) {
        a = take_event(ctx);
        b = take_event(ctx);
        if (!a || !b) {
            if (a) ctx->event_pool.push_back(a);
            if (b) ctx->event_pool.push_back(b);
            a = b = nullptr;
        }
        if (a) RMB_HIP(ctx, hipEventRecord(a, s));
    }
    RMB_HIP(ctx, launch_pair_sym(precision, wall, B, jobs, n_jobs, n_tiles, s));
    if (a) {
        RMB_HIP(ctx, hipEventRecord(b, s));
        ctx->pending.push_back({kid, a, b});
    }
    return RMB_OK;
}

void resolve_timing(rmb_ctx ctx, bool wait) {
    size_t keep = 0;
    for (size_t i = 0; i < ctx->pending.size(); ++i) {
        auto &p = ctx->pending[i];
        if (wait) (void)hipEventSynchronize(p.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ctx->kernel_ms[p.kernel] += ms;
            ctx->kernel_launches[p.kernel] += 1;
            ctx->event_pool.push_back(p.a);
            ctx->event_pool.push_back(p.b);
        } else {
            (void)hipGetLastError();
            ctx->pending[keep++] = p;
        }
    }
    ctx->pending.resize(keep);
}

}  // namespace rmb

using namespace rmb;

extern "C" {

const char *rmb_version(void) { return "rmb 0.1 (gfx950)"; }

// Device address of this device's copy of `scratch`, looked up once per
// device (the device must be current).  Null if the lookup failed.
static void *noalloc_work_address(int device) {
    static std::mutex mu;
    static std::vector<void *> addr;
    static std::vector<bool> tried;
    std::lock_guard<std::mutex> lock(mu);
    if ((size_t)device >= addr.size()) addr.resize(device + 1, nullptr), tried.resize(device + 1, false);
    if (!tried[device]) {
        tried[device] = true;
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) addr[device] = p;
        else (void)hipGetLastError();
    }
    return addr[device];
}

rmb_status rmb_ctx_create(int device, size_t hbm_budget_bytes, rmb_ctx *out) {
    if (!out) return RMB_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return RMB_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return RMB_EDEVICE;
    rmb_ctx c = new rmb_ctx_s();
    c->device = device;
    c->arena = new Arena(hbm_budget_bytes ? hbm_budget_bytes : (size_t(16) << 30));
    c->noalloc_work = noalloc_work_address(device);
    if (const char *e = getenv("RMB_SYM_BAND_BYTES"); e && *e) {
        char *end = nullptr;
        const unsigned long long v = strtoull(e, &end, 10);
        if (end && *end == 0 && v > 0) c->sym_band_bytes = (size_t)v;
    }
    load_tune_cache(c);
    *out = c;
    return RMB_OK;
}

rmb_status rmb_pair_plan(int64_t nb, int32_t *symmetric, int32_t *block) {
    if (nb < 1 || !symmetric || !block) return RMB_EINVAL;
    if (use_sym(nb)) {
        int32_t B, T;
        sym_plan(nb, &B, &T);
        *symmetric = 1;
        *block = B;
    } else {
        int32_t S, Tb;
        int64_t chunk;
        split_plan(nb, &S, &chunk, &Tb);
        *symmetric = 0;
        *block = S;
    }
    return RMB_OK;
}

rmb_status rmb_ctx_set_timing(rmb_ctx ctx, int32_t enable) {
    if (!ctx) return RMB_EINVAL;
    RMB_HIP(ctx, hipSetDevice(ctx->device));
    resolve_timing(ctx, true);
    ctx->timing = enable != 0;
    for (int k = 0; k < RMB_KERNEL_COUNT; ++k) ctx->kernel_ms[k] = 0.0, ctx->kernel_launches[k] = 0;
    return RMB_OK;
}

rmb_status rmb_ctx_kernel_time(rmb_ctx ctx, int32_t kernel, double *total_ms, int64_t *launches) {
    if (!ctx || !total_ms || !launches) return RMB_EINVAL;
    if (kernel < 0 || kernel >= RMB_KERNEL_COUNT) return fail(ctx, RMB_EINVAL, "unknown kernel id %d", kernel);
    RMB_HIP(ctx, hipSetDevice(ctx->device));
    resolve_timing(ctx, true);
    *total_ms = ctx->kernel_ms[kernel];
    *launches = ctx->kernel_launches[kernel];
    return RMB_OK;
}

void rmb_ctx_destroy(rmb_ctx ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    resolve_timing(ctx, true);
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (auto &b : ctx->pinned_cache) (void)hipHostFree(b.first);
    delete ctx->arena;
    delete ctx;
}

const char *rmb_last_error(rmb_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// Workspace of one standalone product, from its base (device, 256-byte
// aligned): [flag | job records, 256 bytes each | partials (symmetric:
// vpart then upart of the largest band) or packed sources then per-split
// partials (one-sided)].
static size_t product_work_bytes(int64_t nb, int32_t precision, size_t band_bytes) {
    if (use_sym(nb)) {
        const size_t jobs = sym_bands(nb, band_bytes).size();
        return 256 + 256 * jobs + sym_band_partial_doubles(nb, band_bytes) * sizeof(double);
    }
    const size_t rec = precision == RMB_PREC_FP32_PAIRS ? sizeof(SrcF32) : sizeof(SrcF64);
    int32_t S, Tb;
    int64_t chunk;
    split_plan(nb, &S, &chunk, &Tb);
    return 512 + (nb * rec + 255) / 256 * 256 + (size_t)S * nb * 3 * sizeof(double);
}

// Enqueues vel = M lambda on `s` with the workspace at `work` (positions
// already validated).  Job records are written by kernels, so nothing here
// allocates or stages host memory.  `timed`: bracket the pair launches with
// the context's timing events when timing is on.
static rmb_status product_enqueue(rmb_ctx ctx, const rmb_system *sys, int32_t precision, const double *lambda,
                                  double *vel, char *work, size_t band_bytes, bool timed, hipStream_t s) {
    const int64_t nb = sys->n_blobs;
    const bool wall = sys->geometry == RMB_GEOM_WALL;
    const double pref = mobility_prefactor(sys->a, sys->eta);
    if (use_sym(nb)) {
        // the symmetric kernel reads positions and forces directly; the
        // output doubles as the accumulator of the bands
        const std::vector<SymBand> bands = sym_bands(nb, band_bytes);
        SymJob J{};
        sym_plan(nb, &J.B, &J.n_blk);
        double *part = (double *)(work + 256 + 256 * bands.size());
        J.tpos = sys->pos;
        J.lam = lambda;
        J.vpart = part;
        J.upart = part + sym_band_partial_doubles(nb, band_bytes) / 2;
        J.vel = vel;
        J.acc = vel;
        J.nb = nb;
        J.a = sys->a;
        J.pref = pref;
        J.f32 = precision == RMB_PREC_FP32_PAIRS;
        for (size_t b = 0; b < bands.size(); ++b) {
            SymJob Jb = J;
            Jb.t0 = bands[b].t0;
            Jb.I0 = bands[b].I0, Jb.I1 = bands[b].I1;
            Jb.first = b == 0, Jb.last = b + 1 == bands.size();
            SymJob *d = (SymJob *)(work + 256 + 256 * b);
            RMB_HIP(ctx, launch_store_sym_job(Jb, d, s));
            if (timed) RMB_TRY(sym_launch(ctx, precision, wall, J.B, d, 1, bands[b].tiles, s));
            else RMB_HIP(ctx, launch_pair_sym(precision, wall, J.B, d, 1, bands[b].tiles, s));
            RMB_HIP(ctx, launch_sym_reduce(d, 1, sym_reduce_groups_band(nb, J.B, bands[b], Jb.last), nullptr, 0, 0, s));
        }
        RMB_HIP(ctx, launch_add_shift(sys->blob_shift, lambda, nb, vel, s));
        return RMB_OK;
    }
    const size_t rec = precision == RMB_PREC_FP32_PAIRS ? sizeof(SrcF32) : sizeof(SrcF64);
    PairJob J;
    pair_job_init(&J, sys->pos, nullptr, nullptr, nb, sys->a);
    const size_t off_src = 512, off_part = off_src + (nb * rec + 255) / 256 * 256;
    J.src = work + off_src;
    J.partial = (double *)(work + off_part);
    J.tile_begin = 0;
    PairJob *d = (PairJob *)(work + 256);
    RMB_HIP(ctx, launch_store_pair_job(J, d, s));
    RMB_HIP(ctx, launch_pack_sources(precision, sys->pos, lambda, nb, work + off_src, s));
    if (timed) RMB_TRY(pair_launch(ctx, precision, wall, d, 1, (int64_t)J.n_tblock * J.n_split, s));
    else RMB_HIP(ctx, launch_pair_tiles(precision, wall, d, 1, (int64_t)J.n_tblock * J.n_split, s));
    RMB_HIP(ctx, launch_reduce_partials(J.partial, J.n_split, nb, pref, vel, s));
    RMB_HIP(ctx, launch_add_shift(sys->blob_shift, lambda, nb, vel, s));
    return RMB_OK;
}

static rmb_status check_product_args(rmb_ctx ctx, const rmb_system *sys, int32_t precision, const double *lambda,
                                     const double *vel) {
    RMB_TRY(check_system(ctx, sys, false));
    if (precision != RMB_PREC_FP64 && precision != RMB_PREC_FP32_PAIRS)
        return fail(ctx, RMB_EINVAL, "unknown precision %d", precision);
    if (!lambda || !vel) return fail(ctx, RMB_EINVAL, "lambda and vel are required");
    if ((const void *)lambda == (const void *)vel) return fail(ctx, RMB_EINVAL, "vel must not alias lambda");
    return RMB_OK;
}

rmb_status rmb_mobility_matvec(rmb_ctx ctx, const rmb_system *sys, int32_t precision, const double *lambda,
                               double *vel, rmb_stream stream) {
    if (!ctx) return RMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    RMB_TRY(check_product_args(ctx, sys, precision, lambda, vel));
    char *base = nullptr;
    RMB_TRY(ctx_scratch(ctx, product_work_bytes(sys->n_blobs, precision, ctx->sym_band_bytes), (void **)&base));
    RMB_TRY(check_positions(ctx, sys, (int *)base, s));
    return product_enqueue(ctx, sys, precision, lambda, vel, base, ctx->sym_band_bytes, true, s);
}

__global__ void zero_flag_kernel(int *flag) { *as_global(flag) = 0; }

// FP32 forces in and velocities out around the FP32-pair product: widening
// to FP64 is exact, and the FP64 sums are rounded to FP32 once at the end.
__global__ void widen_f32_kernel(const float *__restrict__ x, double *__restrict__ y, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) as_global(y)[e] = (double)as_global(x)[e];
}
__global__ void narrow_f64_kernel(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) as_global(y)[e] = (float)as_global(x)[e];
}

rmb_status rmb_mobility_matvec_f32(rmb_ctx ctx, const rmb_system *sys, const float *lambda, float *vel,
                                   rmb_stream stream) {
    if (!ctx) return RMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    RMB_TRY(check_system(ctx, sys, false));
    if (!lambda || !vel) return fail(ctx, RMB_EINVAL, "lambda and vel are required");
    if ((const void *)lambda == (const void *)vel) return fail(ctx, RMB_EINVAL, "vel must not alias lambda");
    const int64_t n3 = 3 * sys->n_blobs;
    const size_t work = (product_work_bytes(sys->n_blobs, RMB_PREC_FP32_PAIRS, ctx->sym_band_bytes) + 255) / 256 * 256;
    const size_t vec = ((size_t)n3 * sizeof(double) + 255) / 256 * 256;
    char *base = nullptr;
    RMB_TRY(ctx_scratch(ctx, work + 2 * vec, (void **)&base));
    RMB_TRY(check_positions(ctx, sys, (int *)base, s));
    double *lam64 = (double *)(base + work), *vel64 = (double *)(base + work + vec);
    const unsigned g = (unsigned)((n3 + 255) / 256);
    hipLaunchKernelGGL(widen_f32_kernel, dim3(g), dim3(256), 0, s, lambda, lam64, n3);
    RMB_HIP(ctx, hipGetLastError());
    RMB_TRY(product_enqueue(ctx, sys, RMB_PREC_FP32_PAIRS, lam64, vel64, base, ctx->sym_band_bytes, true, s));
    hipLaunchKernelGGL(narrow_f64_kernel, dim3(g), dim3(256), 0, s, vel64, vel, n3);
    RMB_HIP(ctx, hipGetLastError());
    return RMB_OK;
}

rmb_status rmb_mobility_matvec_noalloc(rmb_ctx ctx, const rmb_system *sys, int32_t precision, const double *lambda,
                                       double *vel, int32_t validate, rmb_stream stream) {
    if (!ctx) return RMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    RMB_TRY(check_product_args(ctx, sys, precision, lambda, vel));
    char *work = (char *)ctx->noalloc_work;
    if (!work) return fail(ctx, RMB_EDEVICE, "the no-allocation workspace is not available on this device");
    const int64_t nb = sys->n_blobs;
    // bands sized so that [flag | a job record per block row at most | the
    // largest band's partials] fits the static workspace
    size_t band_bytes = kNoAllocBytes;
    if (use_sym(nb)) {
        int32_t B, T;
        sym_plan(nb, &B, &T);
        band_bytes = kNoAllocBytes - 256 - 256 * (size_t)T;
        if (256 + 256 * (size_t)T >= kNoAllocBytes)
            return fail(ctx, RMB_EINVAL, "%lld blobs exceed the no-allocation workspace (%zu MiB)", (long long)nb,
                        kNoAllocBytes >> 20);
    }
    const size_t need = product_work_bytes(nb, precision, band_bytes);
    if (need > kNoAllocBytes)
        return fail(ctx, RMB_EINVAL, "%lld blobs need %zu bytes of workspace, more than the %zu MiB of the "
                    "no-allocation entry point", (long long)nb, need, kNoAllocBytes >> 20);
    if (validate) {
        int *flag = (int *)work;
        int h = 0;
        hipLaunchKernelGGL(zero_flag_kernel, dim3(1), dim3(1), 0, s, flag);
        RMB_HIP(ctx, hipGetLastError());
        RMB_HIP(ctx, launch_validate_positions(sys->pos, nb, sys->geometry == RMB_GEOM_WALL, sys->blob_shift, flag, s));
        RMB_HIP(ctx, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        RMB_HIP(ctx, hipStreamSynchronize(s));
        if (h & 1) return fail(ctx, RMB_EINVAL, "non-finite blob position");
        if (h & 2) return fail(ctx, RMB_EINVAL, "a blob has z <= 0 in wall geometry");
        if (h & 32) return fail(ctx, RMB_EINVAL, "blob_shift must be finite and >= 0");
    }
    return product_enqueue(ctx, sys, precision, lambda, vel, work, band_bytes, false, s);
}

size_t rmb_noalloc_workspace_bytes(void) { return kNoAllocBytes; }

rmb_status rmb_flow_field(rmb_ctx ctx, const rmb_system *sys, int32_t precision, const double *lambda,
                          int32_t n_sub, const double *sub_offsets, double tracer_a, int64_t n_targets,
                          const double *targets, double *vel, rmb_stream stream) {
    if (!ctx) return RMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    RMB_TRY(check_system(ctx, sys, false));
    if (precision != RMB_PREC_FP64 && precision != RMB_PREC_FP32_PAIRS)
        return fail(ctx, RMB_EINVAL, "unknown precision %d", precision);
    if (!lambda) return fail(ctx, RMB_EINVAL, "lambda is required");
    if (n_sub < 1 || n_sub > 65536 || !sub_offsets)
        return fail(ctx, RMB_EINVAL, "n_sub must be in [1, 65536] with sub_offsets given");
    for (int32_t k = 0; k < 3 * n_sub; ++k)
        if (!std::isfinite(sub_offsets[k])) return fail(ctx, RMB_EINVAL, "sub_offsets must be finite");
    if (!(tracer_a > 0.0) || !std::isfinite(tracer_a)) return fail(ctx, RMB_EINVAL, "tracer radius must be > 0");
    if (n_targets < 0 || n_targets > (int64_t(1) << 31) / 3) return fail(ctx, RMB_EINVAL, "n_targets out of range");
    if (n_targets == 0) return RMB_OK;
    if (!targets || !vel) return fail(ctx, RMB_EINVAL, "targets and vel are required");
    if ((const void *)vel == (const void *)lambda || (const void *)vel == (const void *)targets)
        return fail(ctx, RMB_EINVAL, "vel must not alias lambda or targets");
    const int64_t nb = sys->n_blobs, ns = nb * (int64_t)n_sub;
    if (ns > (int64_t(1) << 31) / 3) return fail(ctx, RMB_EINVAL, "n_blobs * n_sub is above the supported maximum");

    const size_t rec = precision == RMB_PREC_FP32_PAIRS ? sizeof(SrcF32) : sizeof(SrcF64);
    const bool wall = sys->geometry == RMB_GEOM_WALL;
    PairJob J;
    pair_job_init_rect(&J, targets, n_targets, nullptr, ns, nullptr, tracer_a);
    // scratch layout: [flag | job | offsets | sources | partials]
    const size_t off_job = 256, off_offs = off_job + 256;
    const size_t off_src = off_offs + ((size_t)n_sub * 24 + 255) / 256 * 256;
    const size_t off_part = off_src + ((size_t)ns * rec + 255) / 256 * 256;
    const size_t total = off_part + (size_t)J.n_split * n_targets * 3 * sizeof(double);
    char *base = nullptr;
    RMB_TRY(ctx_scratch(ctx, total, (void **)&base));
    int *flag = (int *)base;
    // targets: finite, and above the wall in wall geometry
    rmb_system tsys = *sys;
    tsys.pos = targets;
    tsys.n_blobs = n_targets;
    tsys.blob_shift = nullptr;
    {
        const rmb_status st = check_positions(ctx, &tsys, flag, s);
        if (st != RMB_OK) return fail(ctx, st, "target points: %s", rmb_last_error(ctx));
    }
    J.src = base + off_src;
    J.partial = (double *)(base + off_part);
    char *h = nullptr;
    RMB_TRY(pinned(ctx, off_src - off_job, (void **)&h));
    memcpy(h, &J, sizeof(PairJob));
    memcpy(h + (off_offs - off_job), sub_offsets, (size_t)n_sub * 24);
    RMB_HIP(ctx, hipMemcpyAsync(base + off_job, h, off_src - off_job, hipMemcpyHostToDevice, s));
    RMB_HIP(ctx, hipMemsetAsync(flag, 0, sizeof(int), s));
    RMB_HIP(ctx, launch_pack_sub_sources(precision, sys->pos, lambda, nb, (const double *)(base + off_offs), n_sub,
                                         sys->a, wall, base + off_src, flag, s));
    RMB_TRY(pair_launch(ctx, precision, wall, (const PairJob *)(base + off_job), 1,
                        (int64_t)J.n_tblock * J.n_split, s));
    RMB_HIP(ctx, launch_reduce_partials(J.partial, J.n_split, n_targets, mobility_prefactor(tracer_a, sys->eta), vel,
                                        s));
    int *hf = nullptr;
    RMB_TRY(pinned(ctx, sizeof(int), (void **)&hf));
    RMB_HIP(ctx, hipStreamSynchronize(s));  // the staging above is reused below
    RMB_HIP(ctx, hipMemcpyAsync(hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    RMB_HIP(ctx, hipStreamSynchronize(s));
    if (*hf & 1) return fail(ctx, RMB_EINVAL, "non-finite blob position");
    if (*hf & 2) return fail(ctx, RMB_EINVAL, "a sub-blob lies at or below the wall (z <= 0)");
    return RMB_OK;
}

}  // extern "C"

// Library context and host-side helpers (internal).
#pragma once

#include <cstdarg>
#include <map>
#include <string>

#include "rmb_common.h"

struct rmb_ctx_s {
    int device = 0;
    std::string err;
    rmb::Arena *arena = nullptr;
    // Scratch reused by every call on this context (grow-only).
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    // Pinned host staging for small uploads/downloads.
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    // Pinned host buffers given back by finished solve engines, lent to the
    // next ones: pinning host memory costs more than several solve steps.
    std::vector<std::pair<void *, size_t>> pinned_cache;
    hipStream_t last_stream = nullptr;
    bool any_stream = false;
    // kernel timing (diagnostics)
    bool timing = false;
    struct Pending {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    double kernel_ms[RMB_KERNEL_COUNT] = {0, 0, 0, 0};
    int64_t kernel_launches[RMB_KERNEL_COUNT] = {0, 0, 0, 0};
    // tile-shape variant of the large-body factorisation, by padded size:
    // chosen by the autotuner (or read from the persisted tuning file when
    // the context was created), and shapes forced by the caller
    std::map<int, int> tuned_panel;
    std::map<int, int> forced_shape;
    struct TuneRecord {
        int Mp, variant;
        float ms;
    };
    std::vector<TuneRecord> tune_log;
    // this device's copy of the no-allocation entry point's static workspace
    // (device address from hipGetSymbolAddress; null if it could not be had)
    void *noalloc_work = nullptr;
    // budget of one band of the symmetric product's tile partials
    // (RMB_SYM_BAND_BYTES at creation)
    size_t sym_band_bytes = rmb::kSymBandBytes;
};

namespace rmb {

rmb_status fail(rmb_ctx ctx, rmb_status st, const char *fmt, ...);

#define RMB_HIP(ctx, call)                                                                    \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::rmb::fail((ctx), RMB_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define RMB_TRY(expr)                   \
    do {                                \
        rmb_status st_ = (expr);        \
        if (st_ != RMB_OK) return st_;  \
    } while (0)

// Makes the context's device current and orders this call after work the
// previous call left on another stream (scratch and staging are reused).
rmb_status enter(rmb_ctx ctx, hipStream_t s);

// Grow-only scratch of at least `bytes` (device).
rmb_status ctx_scratch(rmb_ctx ctx, size_t bytes, void **out);
// Grow-only pinned host staging of at least `bytes`.
rmb_status pinned(rmb_ctx ctx, size_t bytes, void **out);
// A pinned host buffer of at least `bytes` from the context's cache (or a
// new one); NULL if pinning fails.  *got receives its size.  Give it back
// with pinned_give once no work uses it.
void *pinned_lease(rmb_ctx ctx, size_t bytes, size_t *got);
void pinned_give(rmb_ctx ctx, void *p, size_t bytes);

// Host-side checks of a system description.  need_bodies: body_off and q
// must describe n_bodies bodies covering all blobs.
rmb_status check_system(rmb_ctx ctx, const rmb_system *sys, bool need_bodies);

// Device-side checks of positions (finite; z > 0 above a wall).  Uses
// `flag_dev` (one int of device memory) and synchronises `s`.
rmb_status check_positions(rmb_ctx ctx, const rmb_system *sys, int *flag_dev, hipStream_t s);

// Launches the pair kernels for one (precision, geometry) table, bracketed
// by timing events when the context's kernel timing is on.
rmb_status pair_launch(rmb_ctx ctx, int precision, bool wall, const PairJob *jobs, int32_t n_jobs,
                       int64_t n_tiles, hipStream_t s);
// Same for the symmetric pair kernel (block size B).
rmb_status sym_launch(rmb_ctx ctx, int precision, bool wall, int B, const SymJob *jobs, int32_t n_jobs,
                      int64_t n_tiles, hipStream_t s);
// Reads the persisted autotuner choices into the context.
void load_tune_cache(rmb_ctx ctx);
// Accumulates the elapsed time of completed timing events.
void resolve_timing(rmb_ctx ctx, bool wait);

inline double mobility_prefactor(double a, double eta) {
    return 1.0 / (6.0 * 3.14159265358979323846 * eta * a);
}

}  // namespace rmb

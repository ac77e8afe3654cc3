// Solve engine: right-preconditioned GMRES on the saddle-point system
// (eq:saddle_M) with the block-diagonal preconditioner (eq:indef_block_P),
// optional FP32-pair inner cycles inside FP64 iterative refinement, and
// continuous batching of independent systems.
//
// Every admitted system is a state machine advanced once per tick:
//   SETUP  -> build b = [slip; -F], the preconditioner, and normalise b
//   ITER   -> z = P^-1 v_k, w = A z, CGS2 against V[0..k], v_{k+1} = w/|w|
//   FINISH -> x += P^-1 (V y), then r = b - A_64 x (FP64) and normalise r
// A tick launches each kernel once for all systems that need it (tables of
// per-system descriptors, one upload), copies every system's small results
// back in one download, and synchronises the stream once.  The host then
// applies Givens rotations, tests convergence and chooses each system's
// next step.  A system's arithmetic never depends on which other systems
// share a tick: tilings and reduction orders are functions of its own sizes.
#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>

#include "rmb_body.h"
#include "rmb_ctx.h"

using namespace rmb;

struct rmb_precond_s {
    rmb_ctx ctx = nullptr;
    int64_t nb = 0, N = 0;
    int max_m = 0, max_Mp = 0, variant = 0;
    int32_t n_small = 0, n_large = 0;
    char *dbuf = nullptr;
    BodyWork *items_d = nullptr;
    BigBody *bigs_d = nullptr;
    double *factor = nullptr;
    int *flag_d = nullptr;
    // shared reference-shape factors: one factor per shape, per-body rotations
    int32_t n_shapes = 0;
    double *rot_d = nullptr;
};

namespace rmb {

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Waits for an event by polling for up to 2 ms, then blocking: one GMRES
// step takes well under that, and polling avoids the blocking wait's
// wake-up latency on every step.
static hipError_t wait_event(hipEvent_t e) {
    const double t0 = now_s();
    for (;;) {
        const hipError_t r = hipEventQuery(e);
        if (r != hipErrorNotReady) return r;
        if (now_s() - t0 > 2e-3) return hipEventSynchronize(e);
    }
}

// Host-side description of a system's bodies, split into bodies handled in
// LDS and large bodies (padded, MFMA path), with their factor offsets.
struct BodyLists {
    std::vector<BodyWork> small;
    std::vector<BigBody> large;
    int max_m = 0, max_Mp = 0;
};

static void body_items(const rmb_system &sys, const int64_t *off, double *factor, int *flag, BodyLists &out) {
    out.small.clear();
    out.large.clear();
    out.max_m = out.max_Mp = 0;
    int64_t fo = 0;
    const double pref = mobility_prefactor(sys.a, sys.eta);
    for (int64_t p = 0; p < sys.n_bodies; ++p) {
        BodyWork b{};
        b.pos = sys.pos;
        b.q = sys.q + 3 * p;
        b.factor = factor ? factor + fo : nullptr;
        b.blob0 = off[p];
        b.n_blobs = (int32_t)(off[p + 1] - off[p]);
        b.body = (int32_t)p;
        b.wall = sys.geometry == RMB_GEOM_WALL;
        b.shift = sys.blob_shift;
        b.a = sys.a;
        b.pref = pref;
        b.flag = flag;
        fo += factor_doubles(b.n_blobs);
        if (is_large_body(b.n_blobs)) {
            BigBody g{};
            g.w = b;
            g.Mp = (int32_t)padded_dim(b.n_blobs);
            out.large.push_back(g);
            out.max_Mp = std::max(out.max_Mp, g.Mp);
        } else {
            out.small.push_back(b);
            out.max_m = std::max(out.max_m, 3 * b.n_blobs);
        }
    }
}

static void set_flag(BodyLists &L, int *flag) {
    for (auto &b : L.small) b.flag = flag;
    for (auto &g : L.large) g.w.flag = flag;
}

static int64_t factor_total(const int64_t *off, int64_t N) {
    int64_t t = 0;
    for (int64_t p = 0; p < N; ++p) t += factor_doubles(off[p + 1] - off[p]);
    return t;
}

// Largest padded block of the large-body path: its apply keeps Mp x 8
// doubles of right-hand sides in LDS (48 KiB at 768), beside the 8 KiB
// diagonal block (256 blobs per body).
constexpr int kLargeBodyMaxMp = 768;

static rmb_status check_body_sizes(rmb_ctx ctx, const int64_t *off, int64_t N) {
    for (int64_t p = 0; p < N; ++p)
        if (padded_dim(off[p + 1] - off[p]) > kLargeBodyMaxMp)
            return fail(ctx, RMB_EINVAL, "body %lld has %lld blobs; at most %d blobs per body are supported",
                        (long long)p, (long long)(off[p + 1] - off[p]), (kLargeBodyMaxMp - 6) / 3);
    return RMB_OK;
}

// Batches smaller than this are not timed (too few workgroups to show what
// a full batch would do); they always use the default shape, so that their
// factors do not depend on what the context ran before.
constexpr int32_t kTuneMinBodies = 64;
constexpr int kDefaultShape = 0;

// Persisted autotuner choices: one line "arch tag Mp panel row_tiles chunk"
// per padded size, in the file named by RMB_TUNE_CACHE (empty: none), else
// $XDG_CACHE_HOME/rmb/tune.txt or $HOME/.cache/rmb/tune.txt.  Lines of
// another architecture or kernel generation (tag) are ignored, and so are
// shapes the library no longer has.
static const char *kTuneArch = "gfx950";
static const char *kTuneTag = "chol-panel64-fused-1";

static std::string tune_cache_path() {
    if (const char *e = getenv("RMB_TUNE_CACHE")) return e;
    std::string base;
    if (const char *x = getenv("XDG_CACHE_HOME"); x && *x) base = x;
    else if (const char *h = getenv("HOME"); h && *h) base = std::string(h) + "/.cache";
    else return "";
    return base + "/rmb/tune.txt";
}

static int shape_index(int panel, int row_tiles, int chunk) {
    for (int v = 0; v < large_variant_count(); ++v) {
        int p, g, c;
        large_variant_shape(v, &p, &g, &c);
        if (p == panel && g == row_tiles && c == chunk) return v;
    }
    return -1;
}

void load_tune_cache(rmb_ctx ctx) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    char arch[64], tag[64];
    int Mp, p, g, c;
    while (fscanf(f, "%63s %63s %d %d %d %d", arch, tag, &Mp, &p, &g, &c) == 6) {
        const int v = shape_index(p, g, c);
        if (!strcmp(arch, kTuneArch) && !strcmp(tag, kTuneTag) && v >= 0) ctx->tuned_panel[Mp] = v;  // last wins
    }
    fclose(f);
}

static void save_tune_choice(int Mp, int v) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        // create the directory chain (failures only mean nothing is persisted)
        for (size_t i = 1; i <= slash; ++i)
            if (path[i] == '/' || i == slash) (void)mkdir(path.substr(0, i == slash ? slash : i).c_str(), 0755);
    }
    FILE *f = fopen(path.c_str(), "a");
    if (!f) return;
    int p, g, c;
    large_variant_shape(v, &p, &g, &c);
    fprintf(f, "%s %s %d %d %d %d\n", kTuneArch, kTuneTag, Mp, p, g, c);
    fclose(f);
}

// Tile shape of the large-body factorisation for padded size Mp: the shape
// the caller forced; else the default for small batches; else the tuned
// shape (this context's, or the persisted one), timing every candidate on
// the first batch of that size with at least kTuneMinBodies bodies (the
// timings are kept in the context's tune log and the choice is persisted).
static rmb_status build_large(rmb_ctx ctx, const BigBody *items_d, int32_t n, int max_Mp, hipStream_t s,
                              int *variant_out) {
    auto fo = ctx->forced_shape.find(max_Mp);
    auto it = ctx->tuned_panel.find(max_Mp);
    if (fo != ctx->forced_shape.end() || n < kTuneMinBodies || it != ctx->tuned_panel.end()) {
        const int v = fo != ctx->forced_shape.end() ? fo->second
                      : n < kTuneMinBodies          ? kDefaultShape
                                                    : it->second;
        *variant_out = v;
        RMB_HIP(ctx, launch_precond_build_large(items_d, n, max_Mp, v, s));
        return RMB_OK;
    }
    const int nv = large_variant_count();
    float best_ms = 0.f;
    int best = 0;
    hipEvent_t e0, e1;
    RMB_HIP(ctx, hipEventCreate(&e0));
    RMB_HIP(ctx, hipEventCreate(&e1));
    // one untimed build first, so that the first timed shape does not carry
    // the first launch's costs
    RMB_HIP(ctx, launch_precond_build_large(items_d, n, max_Mp, kDefaultShape, s));
    for (int v = 0; v < nv; ++v) {
        RMB_HIP(ctx, hipEventRecord(e0, s));
        RMB_HIP(ctx, launch_precond_build_large(items_d, n, max_Mp, v, s));
        RMB_HIP(ctx, hipEventRecord(e1, s));
        RMB_HIP(ctx, hipEventSynchronize(e1));
        float ms = 0.f;
        RMB_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        ctx->tune_log.push_back({max_Mp, v, ms});
        if (v == 0 || ms < best_ms) best_ms = ms, best = v;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->tuned_panel[max_Mp] = best;
    save_tune_choice(max_Mp, best);
    if (best != nv - 1) RMB_HIP(ctx, launch_precond_build_large(items_d, n, max_Mp, best, s));
    *variant_out = best;
    return RMB_OK;
}

// ---------------------------------------------------------------------------

enum Phase { SETUP, START, ITER, FINISH, RESID, DONE };

struct Job {
    // request
    int64_t tag = 0;
    rmb_system sys{};
    std::vector<int64_t> off;
    // mobility problem: FT in, U_out and lam_out out; resistance problem
    // (resist): FT holds the body velocities U, U_out receives F = K^T lambda
    const double *FT = nullptr, *slip = nullptr;
    double *U_out = nullptr, *lam_out = nullptr;
    bool resist = false;
    double tol = 1e-8, inner_tol = 1e-5;
    // velocity-error control: u_tol bounds ||U - U_exact|| / ||U_exact||;
    // gamma is the measured ratio of that error to the relative residual
    double u_tol = 0.0, gamma = -1.0, tol_eff = 1e-8, rel_start = 1.0;
    bool gamma_weak = false;  // gamma was measured by a cycle that reduced the residual less than 1000-fold
    int prec = RMB_PREC_FP64, m = 100, max_iters = 1000;
    rmb_precond pc = nullptr;  // external factors (not owned) or null
    // sizes
    int64_t nb = 0, N = 0, n = 0, ldv = 0, nseg = 0;
    int32_t nchunk = 1;
    PairJob pj{};
    int max_m = 0;
    size_t bytes = 0;
    // device
    char *dbuf = nullptr;
    int64_t *off_d = nullptr;
    int32_t *blob_body = nullptr;
    void *src = nullptr;
    double *partial = nullptr, *factor = nullptr;
    double *vel = nullptr;  // reduced product of the symmetric kernel
    bool sym = false;
    int32_t symB = 0, symT = 0;
    std::vector<SymBand> bands;  // symmetric product: bands of tile rows
    size_t band_bytes = kSymBandBytes;  // their partials' budget (the context's)
    BodyWork *items_d = nullptr;
    double *x = nullptr, *b = nullptr, *w = nullptr, *z = nullptr, *V = nullptr;
    double *P1 = nullptr, *P2 = nullptr, *P3 = nullptr;
    double *hred = nullptr;
    int slot = -1;
    BodyLists lists;
    BigBody *bigs_d = nullptr;
    int32_t n_small = 0, n_large = 0;
    int max_Mp = 0, variant = 0;
    // state
    Phase phase = SETUP;
    int k = 0, iters = 0, cycles = 0, mv64 = 0, mv32 = 0;
    double bnorm = 0, rel = 1, target = 0;
    bool cycle_fp32 = false;
    bool step_fp32 = false;  // relaxed precision: the next product in FP32
    double est = 0, est_prev = 0;  // the cycle's last two residual estimates
    std::vector<double> R, cs, sn, g, y;
    rmb_status status = RMB_OK;
    std::string msg;
    double t_admit = 0, t_done = 0;
};

static size_t job_bytes(Job &J) {
    const int64_t nb = J.nb, N = J.N, n = J.n;
    size_t t = 0;
    const size_t part = J.sym ? sym_band_partial_doubles(nb, J.band_bytes) * 8 : (size_t)J.pj.n_split * nb * 24;
    t += al((N + 1) * 8) + al(nb * 4) + al(J.sym ? 0 : nb * sizeof(SrcF64)) + al(part) + al(nb * 24);
    t += 4 * al(n * 8) + al((size_t)(J.m + 1) * J.ldv * 8);
    t += 2 * al((size_t)(J.m + 1) * J.nseg * 8) + al(J.nseg * 8) + al(256 * 8);
    if (!J.pc) t += al(factor_total(J.off.data(), N) * 8) + al(N * sizeof(BodyWork)) + al(N * sizeof(BigBody));
    return t;
}

static void job_carve(Job &J) {
    char *p = J.dbuf;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += al(bytes);
        return r;
    };
    const int64_t nb = J.nb, N = J.N, n = J.n;
    J.off_d = (int64_t *)take((N + 1) * 8);
    J.blob_body = (int32_t *)take(nb * 4);
    J.src = J.sym ? nullptr : take(nb * sizeof(SrcF64));  // packed sources: one-sided kernel only
    J.partial = (double *)take(J.sym ? sym_band_partial_doubles(nb, J.band_bytes) * 8 : (size_t)J.pj.n_split * nb * 24);
    J.vel = (double *)take(nb * 24);
    J.x = (double *)take(n * 8);
    J.b = (double *)take(n * 8);
    J.w = (double *)take(n * 8);
    J.z = (double *)take(n * 8);
    J.V = (double *)take((size_t)(J.m + 1) * J.ldv * 8);
    J.P1 = (double *)take((size_t)(J.m + 1) * J.nseg * 8);
    J.P2 = (double *)take((size_t)(J.m + 1) * J.nseg * 8);
    J.P3 = (double *)take(J.nseg * 8);
    J.hred = (double *)take(256 * 8);
    if (!J.pc) {
        J.factor = (double *)take(factor_total(J.off.data(), N) * 8);
        J.items_d = (BodyWork *)take(N * sizeof(BodyWork));
        J.bigs_d = (BigBody *)take(N * sizeof(BigBody));
    } else {
        J.factor = J.pc->factor;
        J.items_d = J.pc->items_d;
        J.bigs_d = J.pc->bigs_d;
    }
}

// ---------------------------------------------------------------------------

// Host staging of one tick's descriptor tables (pinned), uploaded at once.
struct Staging {
    std::vector<char> host;
    size_t used = 0;
    size_t put(const void *p, size_t bytes) {
        size_t o = (used + 255) / 256 * 256;
        if (host.size() < o + bytes) host.resize(std::max(o + bytes, host.size() * 2 + 4096));
        memcpy(host.data() + o, p, bytes);
        used = o + bytes;
        return o;
    }
    void reset() { used = 0; }
};

struct Engine {
    rmb_ctx ctx;
    hipStream_t s;
    int max_active;
    std::deque<Job *> queue;
    std::vector<Job *> active;
    std::deque<Job *> done;
    // mailbox: per slot, [flag word][hcol: restart + 2 doubles], in pinned
    // host memory, one per tick buffer: the kernels of the tick using buffer
    // `par` write mbox_hp[par] directly, and the host reads it once the
    // tick's event has completed (no copy on the stream)
    static constexpr int kSlot = 260;
    double *mbox_h = nullptr;                 // the host buffer being read
    double *mbox_hp[2] = {nullptr, nullptr};  // one per tick buffer
    int cur = 0;                              // buffer of the tick being enqueued
    size_t mbox_hbytes[2] = {0, 0}, stage_hbytes[2] = {0, 0};  // sizes of the leased host buffers
    hipEvent_t tick_ev[2] = {nullptr, nullptr};  // end of the tick using buffer 0 / 1
    std::vector<int> free_slots;
    // staging
    Staging st;
    char *stage_hp[2] = {nullptr, nullptr}, *stage_d = nullptr;  // host staging, one per tick buffer
    // A lone job in the Arnoldi phase runs one step ahead: the next step is
    // enqueued before the current one's results are read, so the GPU does
    // not wait for the host.  If the current step ends the cycle, the
    // speculative one is ignored (its products are not counted); stream
    // order keeps the work that follows correct.
    bool spec_live = false;
    Job *spec_job = nullptr;
    int spec_k = -1, spec_par = 0, last_par = 1;
    int32_t spec_mv32 = 0, spec_mv64 = 0;
    size_t stage_cap = 0;

    Engine(rmb_ctx c, hipStream_t st_, int maxa) : ctx(c), s(st_), max_active(maxa) {}
    ~Engine() {
        (void)hipStreamSynchronize(s);
        for (Job *j : active) release(j), delete j;
        for (Job *j : queue) delete j;
        for (Job *j : done) delete j;
        for (int b = 0; b < 2; ++b) {
            pinned_give(ctx, mbox_hp[b], mbox_hbytes[b]);
            pinned_give(ctx, stage_hp[b], stage_hbytes[b]);
            if (tick_ev[b]) (void)hipEventDestroy(tick_ev[b]);
        }
        if (stage_d) ctx->arena->free(stage_d);
    }

    rmb_status init() {
        for (int b = 0; b < 2; ++b) {
            mbox_hp[b] = (double *)pinned_lease(ctx, (size_t)max_active * kSlot * 8, &mbox_hbytes[b]);
            if (!mbox_hp[b]) return fail(ctx, RMB_EDEVICE, "pinned host mailbox allocation failed");
            RMB_HIP(ctx, hipEventCreateWithFlags(&tick_ev[b], hipEventDisableTiming));
        }
        mbox_h = mbox_hp[0];
        for (int i = max_active - 1; i >= 0; --i) free_slots.push_back(i);
        return RMB_OK;
    }

    int *flag_d(Job *j) { return (int *)(mbox_hp[cur] + (size_t)j->slot * kSlot); }
    int flag_h(Job *j) { return *(int *)(mbox_h + (size_t)j->slot * kSlot); }
    double *hcol_d(Job *j) { return mbox_hp[cur] + (size_t)j->slot * kSlot + 1; }
    double *hcol_h(Job *j) { return mbox_h + (size_t)j->slot * kSlot + 1; }

    void release(Job *j) {
        if (j->dbuf) {
            ctx->arena->free(j->dbuf);
            stage_reserved -= stage_need(*j);
        }
        j->dbuf = nullptr;
        if (j->slot >= 0) free_slots.push_back(j->slot);
        j->slot = -1;
    }

    rmb_status submit(const rmb_system *sys, const double *FT, const double *slip, double *U, double *lam,
                      const rmb_solve_opts *o, rmb_precond pc, int64_t tag, Job **out, bool resist = false) {
        RMB_TRY(check_system(ctx, sys, true));
        if (!FT || !U || !lam)
            return fail(ctx, RMB_EINVAL, resist ? "U, F and lambda are required" : "FT, U and lambda are required");
        RMB_TRY(check_body_sizes(ctx, sys->body_off, sys->n_bodies));
        auto J = std::make_unique<Job>();
        J->tag = tag;
        J->sys = *sys;
        J->off.assign(sys->body_off, sys->body_off + sys->n_bodies + 1);
        J->sys.body_off = J->off.data();
        J->FT = FT, J->slip = slip, J->U_out = U, J->lam_out = lam;
        if (o) {
            if (o->tol < 0 || o->inner_tol < 0 || o->restart < 0 || o->restart > 255 || o->max_iters < 0 ||
                !(o->u_tol >= 0.0))
                return fail(ctx, RMB_EINVAL, "bad solve options");
            if (o->u_tol > 0 && resist)
                return fail(ctx, RMB_EINVAL, "u_tol applies to mobility solves only");
            J->u_tol = o->u_tol;
            if (o->precision != RMB_PREC_FP64 && o->precision != RMB_PREC_FP32_PAIRS &&
                o->precision != RMB_PREC_RELAXED)
                return fail(ctx, RMB_EINVAL, "unknown precision %d", o->precision);
            if (o->tol > 0) J->tol = o->tol;
            if (o->inner_tol > 0) J->inner_tol = o->inner_tol;
            if (o->restart > 0) J->m = o->restart;
            if (o->max_iters > 0) J->max_iters = o->max_iters;
            J->prec = o->precision;
        }
        if (pc) {
            if (pc->nb != sys->n_blobs || pc->N != sys->n_bodies)
                return fail(ctx, RMB_EINVAL, "preconditioner was built for a different system");
            J->pc = pc;
        }
        J->resist = resist;
        J->tol_eff = J->tol;
        J->nb = sys->n_blobs, J->N = sys->n_bodies;
        J->n = resist ? 3 * J->nb : 3 * J->nb + 6 * J->N;
        J->ldv = (J->n + 31) / 32 * 32;
        {
            int32_t ns = 0;
            krylov_segments(J->n, &ns, &J->nchunk);
            J->nseg = ns;
        }
        pair_job_init(&J->pj, sys->pos, nullptr, nullptr, J->nb, sys->a);
        J->sym = use_sym(J->nb);
        if (J->sym) {
            sym_plan(J->nb, &J->symB, &J->symT);
            J->band_bytes = ctx->sym_band_bytes;
            J->bands = sym_bands(J->nb, J->band_bytes);
        }
        J->bytes = job_bytes(*J);
        if (J->bytes > ctx->arena->budget())
            return fail(ctx, RMB_ENOMEM, "request needs %zu bytes of device memory, budget is %zu", J->bytes,
                        ctx->arena->budget());
        *out = J.get();
        queue.push_back(J.release());
        return RMB_OK;
    }

    // Admission: first come first served, by device-memory footprint.
    void admit() {
        while (!queue.empty() && (int)active.size() < max_active && !free_slots.empty()) {
            Job *J = queue.front();
            const bool staged = grow_stage(stage_reserved + stage_need(*J));
            void *p = staged ? ctx->arena->alloc(J->bytes) : nullptr;
            if (!p) {
                if (active.empty()) {  // can never fit beside the server's own buffers
                    queue.pop_front();
                    J->status = RMB_ENOMEM;
                    J->msg = "request does not fit the device-memory budget";
                    J->phase = DONE;
                    J->t_admit = J->t_done = now_s();
                    done.push_back(J);
                    continue;
                }
                break;
            }
            queue.pop_front();
            J->dbuf = (char *)p;
            stage_reserved += stage_need(*J);
            job_carve(*J);
            J->slot = free_slots.back();
            free_slots.pop_back();
            J->phase = SETUP;
            J->t_admit = now_s();
            J->pj.src = J->src;
            J->pj.partial = J->partial;
            if (!J->pc) {
                body_items(J->sys, J->off.data(), J->factor, nullptr, J->lists);
                J->n_small = (int32_t)J->lists.small.size();
                J->n_large = (int32_t)J->lists.large.size();
                J->max_m = J->lists.max_m;
                J->max_Mp = J->lists.max_Mp;
            } else {
                J->n_small = J->pc->n_small;
                J->n_large = J->pc->n_large;
                J->max_m = J->pc->max_m;
                J->max_Mp = J->pc->max_Mp;
                J->variant = J->pc->variant;
            }
            active.push_back(J);
        }
    }

    // Grows the staging buffers to at least `bytes` (twice that if it fits).
    // The new buffers are allocated before the old ones are released, so a
    // failed attempt leaves the current buffers in place.  Called only
    // between ticks, when no work reads the old buffers.
    bool grow_stage(size_t bytes) {
        if (bytes <= stage_cap) return true;
        size_t want = std::max<size_t>(bytes * 2, 1 << 20);
        char *d = (char *)ctx->arena->alloc(want);
        if (!d) {
            want = std::max<size_t>(bytes, 1 << 20);
            d = (char *)ctx->arena->alloc(want);
        }
        if (!d) return false;
        char *h[2] = {nullptr, nullptr};
        size_t hb[2] = {0, 0};
        for (int b = 0; b < 2; ++b)
            if (!(h[b] = (char *)pinned_lease(ctx, want, &hb[b]))) {
                if (h[0]) pinned_give(ctx, h[0], hb[0]);
                ctx->arena->free(d);
                return false;
            }
        (void)hipStreamSynchronize(s);  // a tick in flight may still read the old buffers
        if (stage_d) ctx->arena->free(stage_d);
        for (int b = 0; b < 2; ++b) {
            pinned_give(ctx, stage_hp[b], stage_hbytes[b]);
            stage_hp[b] = h[b];
            stage_hbytes[b] = hb[b];
        }
        stage_d = d, stage_cap = want;
        return true;
    }
    rmb_status ensure_stage(size_t bytes) {
        return grow_stage(bytes) ? RMB_OK : fail(ctx, RMB_ENOMEM, "staging buffer does not fit the budget");
    }

    // Upper bound of what one job adds to a tick's descriptor tables: its
    // body records and offsets (setup ticks) and a few kilobytes of per-tick
    // tables and Hessenberg coefficients.  Admission reserves it, so a tick
    // never needs staging that the budget cannot provide.
    static size_t stage_need(const Job &J) {
        return 2 * al(J.N * sizeof(BodyWork)) + al(J.N * sizeof(BigBody)) + al((J.N + 1) * 8) +
               al((size_t)(J.m + 1) * 8) + 8192 + 2 * J.bands.size() * sizeof(SymJob);
    }
    static constexpr size_t kStageFixed = 32768;  // alignment of the shared tables
    size_t stage_reserved = kStageFixed;

    // The velocity-error estimate gamma * rel is itself only approximate:
    // gamma is measured on the residual a cycle started from, and the
    // residual left at the end lies more in the slowly converging directions,
    // which amplify it more.  Solves aim at half the bound when the cycle that
    // measured gamma reduced the residual at least 1000-fold (estimates
    // within 1.2x of the true error), at a quarter after a shorter cycle, such
    // as the tenfold verification cycle (up to 2.2x measured).
    static constexpr double kUtolSafety = 0.5, kUtolSafetyShort = 0.25;
    static double utol_safety(const Job *J) { return J->gamma_weak ? kUtolSafetyShort : kUtolSafety; }

    // Residual target of the next cycle.  Under velocity-error control the
    // solve's tolerance is min(tol, u_tol / gamma) once a refinement cycle
    // has measured gamma; a solve that meets `tol` before any such cycle runs
    // a verification cycle that reduces the residual tenfold.
    void begin_cycle(Job *J, double beta) {
        J->k = 0;
        J->cycles++;
        J->rel_start = beta / J->bnorm;
        J->cycle_fp32 = J->prec == RMB_PREC_FP32_PAIRS;
        J->tol_eff = J->u_tol > 0 && J->gamma > 0 ? std::min(J->tol, utol_safety(J) * J->u_tol / J->gamma) : J->tol;
        double t = J->tol_eff * J->bnorm;
        if (J->u_tol > 0 && !(J->gamma > 0) && beta <= J->tol * J->bnorm) t = 0.1 * beta;
        J->target = J->cycle_fp32 ? std::max(J->inner_tol * beta, 0.5 * t) : t;
        J->step_fp32 = relaxed_fp32(J, beta);
        J->est = beta, J->est_prev = 0;
        J->R.assign((size_t)J->m * J->m, 0.0);
        J->cs.assign(J->m, 0.0);
        J->sn.assign(J->m, 0.0);
        J->g.assign(J->m + 1, 0.0);
        J->g[0] = beta;
        J->phase = ITER;
    }

    // Relaxed precision: an FP32-pair product (relative error below
    // kFp32ProductError) is accurate enough once tol ||b|| / ||r_k|| exceeds
    // that error, ||r_k|| being the current residual (estimate).
    static constexpr double kFp32ProductError = 1e-7;
    static bool relaxed_fp32(const Job *J, double rnorm) {
        return J->prec == RMB_PREC_RELAXED && rnorm * kFp32ProductError <= J->tol_eff * J->bnorm;
    }

    void finish_job(Job *J, rmb_status st, const char *msg) {
        J->status = st;
        if (msg) J->msg = msg;
        J->phase = DONE;
    }

    // ---------------------------------------------------------------------
    // Speculation pays only if the step in flight is unlikely to end the
    // cycle: the residual estimate falls roughly geometrically, so the step
    // is skipped when the last reduction ratio predicts the target within a
    // factor 1.5.
    static bool can_speculate(const Job *J) {
        if (!(J->phase == ITER && J->k + 1 < J->m && J->iters + 1 < J->max_iters &&
              (J->prec != RMB_PREC_RELAXED || J->step_fp32)))
            return false;
        const double rho = J->est_prev > 0 ? J->est / J->est_prev : 1.0;
        return J->est * rho > 1.5 * J->target;
    }

    rmb_status step() {
        if (spec_live) {
            Job *J = spec_job;
            const bool valid = J->phase == ITER && J->k == spec_k;
            if (valid && !(active.size() == 1 && queue.empty())) {
                // other work arrived: finish the step already in flight on its own
                spec_live = false;
                J->mv32 += spec_mv32, J->mv64 += spec_mv64;
                std::vector<Job *> none, it{J};
                RMB_TRY(complete(none, none, it, spec_par));
                return finalize_done();
            }
            if (!valid) spec_live = false;  // ignored; later work is stream-ordered after it
        }
        admit();
        if (active.empty()) return RMB_OK;
        std::vector<Job *> setup, finish, iter;
        for (Job *J : active) {
            if (J->phase == SETUP) setup.push_back(J);
            else if (J->phase == FINISH) finish.push_back(J);
            else if (J->phase == ITER) iter.push_back(J);
        }
        // this tick: the speculative step already in flight, or a new launch
        int par;
        if (spec_live) {
            par = spec_par;
            spec_live = false;
            spec_job->mv32 += spec_mv32, spec_job->mv64 += spec_mv64;
        } else {
            par = 1 - last_par;
            RMB_TRY(launch(setup, finish, iter, par, 0));
            last_par = par;
        }
        // a lone Arnoldi job: enqueue its next step before reading this one
        if (active.size() == 1 && queue.empty() && iter.size() == 1 && can_speculate(iter[0])) {
            std::vector<Job *> none, it{iter[0]};
            spec_mv32 = spec_mv64 = 0;
            RMB_TRY(launch(none, none, it, 1 - par, 1));
            last_par = 1 - par;
            spec_live = true, spec_job = iter[0], spec_k = iter[0]->k + 1, spec_par = 1 - par;
        }
        RMB_TRY(complete(setup, finish, iter, par));
        if (spec_live && !(spec_job->phase == ITER && spec_job->k == spec_k)) spec_live = false;
        return finalize_done();
    }

    // Enqueues one tick for the given jobs: descriptor tables (through host
    // staging buffer `par`) and every launch, whose mailbox writes go to host
    // buffer `par`, followed by tick_ev[par].  koff = 1 builds the
    // Arnoldi jobs' step for index k + 1 (a speculative step; its products
    // are counted apart until it is accepted).
    rmb_status launch(std::vector<Job *> &setup, std::vector<Job *> &finish, std::vector<Job *> &iter, int par,
                      int koff) {
        cur = par;
        st.reset();


        // --- descriptor tables ------------------------------------------
        // precond build items (setup jobs without external factors)
        std::vector<BodyWork> build_items;
        int build_max_m = 0;
        // setup items copies (persistent per job): offsets into staging
        std::vector<size_t> o_items(setup.size(), 0), o_bigs(setup.size(), 0), o_off(setup.size(), 0);
        for (size_t i = 0; i < setup.size(); ++i) {
            Job *J = setup[i];
            if (!J->pc) {
                set_flag(J->lists, flag_d(J));
                for (auto &b : J->lists.small) build_items.push_back(b);
                build_max_m = std::max(build_max_m, J->max_m);
                if (J->n_small) o_items[i] = st.put(J->lists.small.data(), J->n_small * sizeof(BodyWork));
                if (J->n_large) o_bigs[i] = st.put(J->lists.large.data(), J->n_large * sizeof(BigBody));
            }
            o_off[i] = st.put(J->off.data(), J->off.size() * sizeof(int64_t));
        }
        size_t o_build = build_items.empty() ? 0 : st.put(build_items.data(), build_items.size() * sizeof(BodyWork));

        // combine (finish): coefficients y
        std::vector<KrylovJob> comb;
        std::vector<size_t> o_coef;
        int64_t wg_comb = 0;
        for (Job *J : finish) o_coef.push_back(st.put(J->y.data(), J->y.size() * 8));
        // precond apply: finish (z -> w) then iter (V_k -> z)
        std::vector<PrecondApplyJob> app, appL;  // small bodies, large bodies
        int64_t wg_app = 0, wg_appL = 0;
        int app_max_m = 0, appL_max_Mp = 0;
        auto add_app = [&](Job *J, const double *in, double *out) {
            PrecondApplyJob a{};
            a.in = in;
            a.out = out;
            a.ld = J->n;
            a.nb3 = 3 * J->nb;
            a.nrhs = 1;
            a.mode = J->resist ? 1 : 0;
            if (J->n_small) {
                a.items = J->items_d;
                a.wg_begin = wg_app;
                a.n_items = J->n_small;
                app.push_back(a);
                wg_app += J->n_small;
                app_max_m = std::max(app_max_m, J->max_m);
            }
            if (J->n_large) {
                a.items = (const BodyWork *)J->bigs_d;
                a.wg_begin = wg_appL;
                a.n_items = J->n_large;
                appL.push_back(a);
                wg_appL += J->n_large;
                appL_max_Mp = std::max(appL_max_Mp, J->max_Mp);
            }
        };
        for (Job *J : finish) add_app(J, J->z, J->w);
        for (Job *J : iter) add_app(J, J->V + (size_t)(J->k + koff) * J->ldv, J->z);

        // matvec operands: iter (z, its cycle precision), finish/resid (x, FP64)
        std::vector<Job *> mv = iter;
        for (Job *J : finish) mv.push_back(J);
        std::vector<PackJob> pk;
        int64_t wg_pk = 0;
        std::vector<PairJob> pairs[2][2];  // [fp32][wall]
        int64_t tiles[2][2] = {{0, 0}, {0, 0}};
        // symmetric product, per band index: tile tables [fp32][wall][block
        // size 64/128/256] and the reduction table of the systems with that band
        struct BandTables {
            std::vector<SymJob> syms[2][2][3];
            int64_t stiles[2][2][3] = {};
            size_t o_sym[2][2][3] = {};
            std::vector<SymJob> sred;
            int64_t wg_sred = 0;
            size_t o_sred = 0;
        };
        std::vector<BandTables> bt;
        auto bidx = [](int B) { return B == 64 ? 0 : B == 128 ? 1 : 2; };
        std::vector<SaddleJob> sd;
        int64_t wg_sd_blob = 0, wg_sd_body = 0;
        for (Job *J : mv) {
            const bool is_iter = J->phase == ITER;
            const bool f32 = is_iter && (J->cycle_fp32 || J->step_fp32);
            const double *xin = is_iter ? J->z : J->x;
            if (!J->sym) {  // the symmetric kernel reads positions and forces directly
                PackJob p{};
                p.pos = J->sys.pos;
                p.lam = xin;
                p.src = J->src;
                p.nb = J->nb;
                p.wg_begin = wg_pk;
                p.precision = f32 ? RMB_PREC_FP32_PAIRS : RMB_PREC_FP64;
                pk.push_back(p);
                wg_pk += (J->nb + 255) / 256;
            }
            const int wl = J->sys.geometry == RMB_GEOM_WALL;
            if (J->sym) {
                SymJob y{};
                y.tpos = J->sys.pos;
                y.lam = xin;
                y.vpart = J->partial;
                y.upart = J->partial + sym_band_partial_doubles(J->nb, J->band_bytes) / 2;
                y.vel = J->vel;
                y.acc = J->vel;  // unused by the product otherwise (the reduction writes the saddle rows)
                y.nb = J->nb;
                y.n_blk = J->symT;
                y.B = J->symB;
                y.a = J->sys.a;
                y.pref = mobility_prefactor(J->sys.a, J->sys.eta);
                y.f32 = f32 ? 1 : 0;
                const int bi = bidx(J->symB);
                y.epi = (const void *)(uintptr_t)sd.size();  // index of its saddle rows; patched below
                const int nband = (int)J->bands.size();
                if ((int)bt.size() < nband) bt.resize(nband);
                for (int b = 0; b < nband; ++b) {
                    const SymBand &band = J->bands[b];
                    BandTables &T = bt[b];
                    y.t0 = band.t0;
                    y.I0 = band.I0, y.I1 = band.I1;
                    y.first = b == 0, y.last = b == nband - 1;
                    y.wg_begin = T.stiles[f32][wl][bi];
                    y.red_begin = T.wg_sred;
                    T.stiles[f32][wl][bi] += band.tiles;
                    T.wg_sred += sym_reduce_groups_band(J->nb, J->symB, band, y.last);
                    T.syms[f32][wl][bi].push_back(y);
                    T.sred.push_back(y);
                }
            } else {
                PairJob pj = J->pj;
                pj.tile_begin = tiles[f32][wl];
                pairs[f32][wl].push_back(pj);
                tiles[f32][wl] += (int64_t)pj.n_tblock * pj.n_split;
            }
            SaddleJob sj{};
            sj.pos = J->sys.pos;
            sj.q = J->sys.q;
            sj.body_off = J->off_d;
            sj.blob_body = J->blob_body;
            sj.partial = J->sym ? J->vel : J->partial;
            sj.x = xin;
            sj.b = is_iter ? nullptr : J->b;
            sj.shift = J->sys.blob_shift;
            sj.y = J->w;
            sj.nb = J->nb;
            sj.blk_begin = wg_sd_blob;
            sj.body_begin = wg_sd_body;
            sj.n_split = J->sym ? 1 : J->pj.n_split;
            sj.resist = J->resist ? 1 : 0;
            sj.pref = J->sym ? 1.0 : mobility_prefactor(J->sys.a, J->sys.eta);
            sd.push_back(sj);
            wg_sd_blob += J->sym ? 0 : (J->nb + 255) / 256;  // symmetric: rows written by the reduction
            wg_sd_body += J->resist ? 0 : J->N;
            if (koff) (f32 ? spec_mv32 : spec_mv64)++;
            else if (f32) J->mv32++; else J->mv64++;
        }

        // orthogonalisation / normalisation: iter (kk = k+1), finish->resid
        // and setup->start (kk = 0)
        std::vector<KrylovJob> orth;
        int64_t wg_orth = 0;
        auto kj = [&](Job *J, double *w, int kk, double *vnext, int64_t &wg) {
            KrylovJob K{};
            K.V = J->V;
            K.ldv = J->ldv;
            K.w = w;
            K.vnext = vnext;
            K.P1 = J->P1;
            K.P2 = J->P2;
            K.P3 = J->P3;
            K.hcol = hcol_d(J);
            K.hred = J->hred;
            K.n = J->n;
            K.wg_begin = wg;
            K.n_seg = (int32_t)J->nseg;
            K.n_chunk = J->nchunk;
            K.kk = kk;
            wg += J->nseg;
            return K;
        };
        for (Job *J : iter)
            orth.push_back(kj(J, J->w, J->k + koff + 1, J->V + (size_t)(J->k + koff + 1) * J->ldv, wg_orth));
        for (Job *J : finish) orth.push_back(kj(J, J->w, 0, J->V, wg_orth));
        // velocity norms of the correction and the updated iterate (after the axpy)
        std::vector<KrylovJob> un;
        for (Job *J : finish)
            if (J->u_tol > 0) {
                int64_t unused = 0;
                KrylovJob U = kj(J, nullptr, 0, nullptr, unused);
                U.wg_begin = (int64_t)un.size();  // one workgroup per job
                U.x = J->x;
                U.t = J->w;
                U.u0 = 3 * J->nb;
                un.push_back(U);
            }
        for (Job *J : setup) orth.push_back(kj(J, J->b, 0, J->V, wg_orth));
        // finish: combine then axpy tables
        std::vector<KrylovJob> axp;
        int64_t wg_axp = 0;
        for (size_t i = 0; i < finish.size(); ++i) {
            Job *J = finish[i];
            KrylovJob K = kj(J, J->z, (int)J->y.size(), nullptr, wg_comb);
            K.coef = (const double *)(uintptr_t)o_coef[i];  // patched below
            comb.push_back(K);
            KrylovJob A = kj(J, nullptr, 0, nullptr, wg_axp);
            A.x = J->x;
            A.t = J->w;
            axp.push_back(A);
        }

        size_t o_app = app.empty() ? 0 : st.put(app.data(), app.size() * sizeof(PrecondApplyJob));
        size_t o_appL = appL.empty() ? 0 : st.put(appL.data(), appL.size() * sizeof(PrecondApplyJob));
        size_t o_pk = pk.empty() ? 0 : st.put(pk.data(), pk.size() * sizeof(PackJob));
        size_t o_pair[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                o_pair[a][b] = pairs[a][b].empty() ? 0 : st.put(pairs[a][b].data(), pairs[a][b].size() * sizeof(PairJob));
        size_t n_sred = 0;
        for (BandTables &T : bt) {
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int c = 0; c < 3; ++c)
                        if (!T.syms[a][b][c].empty())
                            T.o_sym[a][b][c] = st.put(T.syms[a][b][c].data(), T.syms[a][b][c].size() * sizeof(SymJob));
            n_sred += T.sred.size();
        }
        size_t o_sd = sd.empty() ? 0 : st.put(sd.data(), sd.size() * sizeof(SaddleJob));
        size_t o_orth = orth.empty() ? 0 : st.put(orth.data(), orth.size() * sizeof(KrylovJob));
        size_t o_axp = axp.empty() ? 0 : st.put(axp.data(), axp.size() * sizeof(KrylovJob));
        size_t o_un = un.empty() ? 0 : st.put(un.data(), un.size() * sizeof(KrylovJob));
        // the combine and reduction tables hold device addresses inside the
        // staging buffer (coefficients, saddle rows): patched once it is sized
        size_t o_comb = 0;
        RMB_TRY(ensure_stage(st.used + comb.size() * sizeof(KrylovJob) + n_sred * sizeof(SymJob) + 8192 +
                             256 * bt.size()));
        for (auto &K : comb) K.coef = (const double *)(stage_d + (size_t)(uintptr_t)K.coef);
        if (!comb.empty()) o_comb = st.put(comb.data(), comb.size() * sizeof(KrylovJob));
        for (BandTables &T : bt) {
            for (auto &y : T.sred) y.epi = stage_d + o_sd + (size_t)(uintptr_t)y.epi * sizeof(SaddleJob);
            if (!T.sred.empty()) T.o_sred = st.put(T.sred.data(), T.sred.size() * sizeof(SymJob));
        }
        RMB_TRY(ensure_stage(st.used));
        memcpy(stage_hp[par], st.host.data(), st.used);
        RMB_HIP(ctx, hipMemcpyAsync(stage_d, stage_hp[par], st.used, hipMemcpyHostToDevice, s));
        auto D = [&](size_t o) { return (void *)(stage_d + o); };

        // --- launches -------------------------------------------------------
        for (size_t i = 0; i < setup.size(); ++i) {
            Job *J = setup[i];
            RMB_HIP(ctx, hipMemsetAsync(flag_d(J), 0, sizeof(int), s));
            RMB_HIP(ctx, launch_validate_positions(J->sys.pos, J->nb, J->sys.geometry == RMB_GEOM_WALL,
                                                   J->sys.blob_shift, flag_d(J), s));
            RMB_HIP(ctx, hipMemcpyAsync(J->off_d, D(o_off[i]), J->off.size() * 8, hipMemcpyDeviceToDevice, s));
            if (!J->pc && J->n_small)
                RMB_HIP(ctx, hipMemcpyAsync(J->items_d, D(o_items[i]), J->n_small * sizeof(BodyWork),
                                            hipMemcpyDeviceToDevice, s));
            if (!J->pc && J->n_large)
                RMB_HIP(ctx, hipMemcpyAsync(J->bigs_d, D(o_bigs[i]), J->n_large * sizeof(BigBody),
                                            hipMemcpyDeviceToDevice, s));
            RMB_HIP(ctx, launch_blob_body(J->off_d, J->N, J->blob_body, s));
            if (J->resist)
                RMB_HIP(ctx, launch_build_rhs_resist(J->FT, J->slip, J->sys.pos, J->sys.q, J->blob_body, J->nb, J->b,
                                                     s));
            else
                RMB_HIP(ctx, launch_build_rhs(J->FT, J->slip, J->nb, J->N, J->b, s));
            RMB_HIP(ctx, hipMemsetAsync(J->x, 0, J->n * 8, s));
        }
        if (!build_items.empty())
            RMB_HIP(ctx, launch_precond_build_small((const BodyWork *)D(o_build), (int32_t)build_items.size(),
                                                    build_max_m, s));
        for (Job *J : setup)
            if (!J->pc && J->n_large) RMB_TRY(build_large(ctx, J->bigs_d, J->n_large, J->max_Mp, s, &J->variant));
        if (!comb.empty()) RMB_HIP(ctx, launch_combine((const KrylovJob *)D(o_comb), (int32_t)comb.size(), wg_comb, s));
        if (!app.empty())
            RMB_HIP(ctx, launch_precond_apply_small((const PrecondApplyJob *)D(o_app), (int32_t)app.size(), wg_app, 1,
                                                    app_max_m, s));
        if (!appL.empty())
            RMB_HIP(ctx, launch_precond_apply_large((const PrecondApplyJob *)D(o_appL), (int32_t)appL.size(), wg_appL, 1,
                                                    appL_max_Mp, s));
        if (!axp.empty()) RMB_HIP(ctx, launch_axpy((const KrylovJob *)D(o_axp), (int32_t)axp.size(), wg_axp, s));
        if (!un.empty()) RMB_HIP(ctx, launch_unorm((const KrylovJob *)D(o_un), (int32_t)un.size(), s));
        if (!pk.empty()) RMB_HIP(ctx, launch_pack_table((const PackJob *)D(o_pk), (int32_t)pk.size(), wg_pk, s));
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                if (!pairs[a][b].empty())
                    RMB_TRY(pair_launch(ctx, a ? RMB_PREC_FP32_PAIRS : RMB_PREC_FP64, b != 0,
                                        (const PairJob *)D(o_pair[a][b]), (int32_t)pairs[a][b].size(), tiles[a][b], s));
        {
            const int Bs[3] = {64, 128, 256};
            for (size_t band = 0; band < bt.size(); ++band) {
                BandTables &T = bt[band];
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 3; ++c)
                            if (!T.syms[a][b][c].empty())
                                RMB_TRY(sym_launch(ctx, a ? RMB_PREC_FP32_PAIRS : RMB_PREC_FP64, b != 0, Bs[c],
                                                   (const SymJob *)D(T.o_sym[a][b][c]),
                                                   (int32_t)T.syms[a][b][c].size(), T.stiles[a][b][c], s));
                // the saddle body rows ride on the first reduction launch
                RMB_HIP(ctx, launch_sym_reduce((const SymJob *)D(T.o_sred), (int32_t)T.sred.size(), T.wg_sred,
                                               band == 0 && !sd.empty() ? (const SaddleJob *)D(o_sd) : nullptr,
                                               (int32_t)sd.size(), band == 0 ? wg_sd_body : 0, s));
            }
            if (!bt.empty()) wg_sd_body = 0;
        }
        if (!sd.empty())
            RMB_HIP(ctx, launch_saddle((const SaddleJob *)D(o_sd), (int32_t)sd.size(), wg_sd_blob, wg_sd_body, s));
        if (!orth.empty())
            RMB_HIP(ctx, launch_orthogonalise((const KrylovJob *)D(o_orth), (int32_t)orth.size(), wg_orth, s));
        RMB_HIP(ctx, hipEventRecord(tick_ev[par], s));
        return RMB_OK;
    }

    // Waits for the tick that used buffer `par` and applies its results on
    // the host (Givens rotations, convergence tests, next phases).
    rmb_status complete(std::vector<Job *> &setup, std::vector<Job *> &finish, std::vector<Job *> &iter, int par) {
        RMB_HIP(ctx, wait_event(tick_ev[par]));
        mbox_h = mbox_hp[par];
        // timed launches are resolved in batches (each query costs host
        // time that would otherwise delay the next tick's launches)
        if (ctx->timing && ctx->pending.size() >= 512) resolve_timing(ctx, false);

        // --- host updates -------------------------------------------------
        for (Job *J : setup) {
            const int f = flag_h(J);
            if (f & 3) { finish_job(J, RMB_EINVAL, (f & 1) ? "non-finite blob position" : "a blob has z <= 0 in wall geometry"); continue; }
            if (f & 32) { finish_job(J, RMB_EINVAL, "blob_shift must be finite and >= 0"); continue; }
            if (f & 4) { finish_job(J, RMB_ENOTSPD, "a body's mobility block is not positive definite"); continue; }
            // the resistance problem uses M_pp^-1 alone
            if ((f & 8) && !J->resist) { finish_job(J, RMB_ENOTSPD, "a body's K^T M^-1 K block is singular"); continue; }
            J->bnorm = hcol_h(J)[0];
            if (!(J->bnorm > 0.0)) {
                J->rel = 0.0;
                finish_job(J, RMB_OK, nullptr);  // x = 0 solves b = 0
                continue;
            }
            J->rel = 1.0;
            begin_cycle(J, J->bnorm);
        }
        for (Job *J : finish) {
            const double beta = hcol_h(J)[0];
            J->rel = beta / J->bnorm;
            bool ok = J->rel <= J->tol;
            if (J->u_tol > 0) {
                // the cycle's correction d estimates the error of the iterate it
                // started from, whose relative residual was rel_start
                const double du = std::sqrt(hcol_h(J)[1]), xu = std::sqrt(hcol_h(J)[2]);
                if (J->cycles >= 2 && J->rel_start > 0 && xu > 0) {
                    J->gamma = du / xu / J->rel_start;
                    J->gamma_weak = J->rel > 1e-3 * J->rel_start;
                }
                ok = ok && J->gamma > 0 && J->gamma * J->rel <= utol_safety(J) * J->u_tol;
            }
            if (ok) finish_job(J, RMB_OK, nullptr);
            else if (J->iters >= J->max_iters) finish_job(J, RMB_ENOCONV, "iteration limit reached");
            else begin_cycle(J, beta);
        }
        for (Job *J : iter) {
            const double *h = hcol_h(J);
            const int k = J->k;
            std::vector<double> c(h, h + k + 2);
            for (int i = 0; i < k; ++i) {
                const double t = J->cs[i] * c[i] + J->sn[i] * c[i + 1];
                c[i + 1] = -J->sn[i] * c[i] + J->cs[i] * c[i + 1];
                c[i] = t;
            }
            const double den = std::hypot(c[k], c[k + 1]);
            bool breakdown = !(den > 0.0);
            if (!breakdown) {
                J->cs[k] = c[k] / den;
                J->sn[k] = c[k + 1] / den;
                c[k] = den;
                J->g[k + 1] = -J->sn[k] * J->g[k];
                J->g[k] = J->cs[k] * J->g[k];
            }
            for (int i = 0; i <= k; ++i) J->R[(size_t)i * J->m + k] = c[i];
            J->k = k + 1;
            J->iters++;
            J->step_fp32 = relaxed_fp32(J, std::fabs(J->g[J->k]));
            J->est_prev = J->est, J->est = std::fabs(J->g[J->k]);
            const bool lucky = !(h[k + 1] > 1e-300 * std::max(1.0, J->bnorm));
            if (breakdown || lucky || std::fabs(J->g[J->k]) <= J->target || J->k >= J->m || J->iters >= J->max_iters) {
                // y = R^-1 g over the first kk columns (drop a singular last column)
                int kk = J->k;
                if (breakdown) kk = J->k - 1;
                J->y.assign(kk, 0.0);
                for (int i = kk - 1; i >= 0; --i) {
                    double v = J->g[i];
                    for (int j = i + 1; j < kk; ++j) v -= J->R[(size_t)i * J->m + j] * J->y[j];
                    J->y[i] = v / J->R[(size_t)i * J->m + i];
                }
                J->phase = FINISH;
            }
        }

        return RMB_OK;
    }

    // Hands finished jobs back: outputs copied, stream drained (a
    // speculative step may still be running), buffers released.
    rmb_status finalize_done() {
        std::vector<Job *> fin;
        for (Job *J : active)
            if (J->phase == DONE) fin.push_back(J);
        if (!fin.empty()) {
            for (Job *J : fin) {
                if (J->status == RMB_OK || J->status == RMB_ENOCONV) {
                    RMB_HIP(ctx, hipMemcpyAsync(J->lam_out, J->x, 3 * J->nb * 8, hipMemcpyDeviceToDevice, s));
                    if (J->resist)
                        RMB_HIP(ctx, launch_body_forces(J->sys.pos, J->sys.q, J->off_d, J->x, J->N, J->U_out, s));
                    else
                        RMB_HIP(ctx, hipMemcpyAsync(J->U_out, J->x + 3 * J->nb, 6 * J->N * 8,
                                                    hipMemcpyDeviceToDevice, s));
                }
            }
            RMB_HIP(ctx, hipStreamSynchronize(s));
            const double t = now_s();
            for (Job *J : fin) {
                J->t_done = t;
                release(J);
                done.push_back(J);
            }
            active.erase(std::remove_if(active.begin(), active.end(), [](Job *J) { return J->phase == DONE; }),
                         active.end());
        }
        return RMB_OK;
    }

    static void fill_info(const Job *J, rmb_solve_info *info) {
        if (!info) return;
        info->status = J->status;
        info->iterations = J->iters;
        info->cycles = J->cycles;
        info->matvecs_fp64 = J->mv64;
        info->matvecs_fp32 = J->mv32;
        info->pad = 0;
        info->rel_residual = J->rel;
        info->seconds = J->t_done - J->t_admit;
        info->tol_internal = J->tol_eff;
        info->gamma = J->gamma > 0 ? J->gamma : -1.0;
        info->u_err_est = J->u_tol > 0 && J->gamma > 0 ? J->gamma * J->rel : -1.0;
    }
};

}  // namespace rmb

struct rmb_server_s {
    rmb::Engine *eng = nullptr;
};

extern "C" {

// ---------------------------------------------------------------------------
// preconditioner entry points
// ---------------------------------------------------------------------------

rmb_status rmb_precond_factor(rmb_ctx ctx, const rmb_system *sys, rmb_precond *out, rmb_stream stream) {
    if (!ctx || !out) return RMB_EINVAL;
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    RMB_TRY(check_system(ctx, sys, true));
    RMB_TRY(check_body_sizes(ctx, sys->body_off, sys->n_bodies));
    auto pc = new rmb_precond_s();
    pc->ctx = ctx;
    pc->nb = sys->n_blobs;
    pc->N = sys->n_bodies;
    const size_t fbytes = al(factor_total(sys->body_off, sys->n_bodies) * 8);
    const size_t ibytes = al(sys->n_bodies * sizeof(BodyWork));
    const size_t gbytes = al(sys->n_bodies * sizeof(BigBody));
    pc->dbuf = (char *)ctx->arena->alloc(fbytes + ibytes + gbytes + 256);
    if (!pc->dbuf) {
        delete pc;
        return fail(ctx, RMB_ENOMEM, "preconditioner factors (%zu bytes) exceed the budget", fbytes + ibytes + gbytes);
    }
    pc->factor = (double *)pc->dbuf;
    pc->items_d = (BodyWork *)(pc->dbuf + fbytes);
    pc->bigs_d = (BigBody *)(pc->dbuf + fbytes + ibytes);
    pc->flag_d = (int *)(pc->dbuf + fbytes + ibytes + gbytes);
    BodyLists lists;
    body_items(*sys, sys->body_off, pc->factor, pc->flag_d, lists);
    pc->n_small = (int32_t)lists.small.size();
    pc->n_large = (int32_t)lists.large.size();
    pc->max_m = lists.max_m;
    pc->max_Mp = lists.max_Mp;
    auto cleanup = [&](rmb_status st) {
        ctx->arena->free(pc->dbuf);
        delete pc;
        return st;
    };
    rmb_status st = check_positions(ctx, sys, pc->flag_d, s);
    if (st != RMB_OK) return cleanup(st);
    const size_t hs = lists.small.size() * sizeof(BodyWork), hl = lists.large.size() * sizeof(BigBody);
    char *h = nullptr;
    st = pinned(ctx, hs + hl + 64, (void **)&h);
    if (st != RMB_OK) return cleanup(st);
    memcpy(h, lists.small.data(), hs);
    memcpy(h + hs, lists.large.data(), hl);
    if (hipMemsetAsync(pc->flag_d, 0, sizeof(int), s) != hipSuccess ||
        (hs && hipMemcpyAsync(pc->items_d, h, hs, hipMemcpyHostToDevice, s) != hipSuccess) ||
        (hl && hipMemcpyAsync(pc->bigs_d, h + hs, hl, hipMemcpyHostToDevice, s) != hipSuccess) ||
        launch_precond_build_small(pc->items_d, pc->n_small, pc->max_m, s) != hipSuccess)
        return cleanup(fail(ctx, RMB_EDEVICE, "preconditioner build launch failed"));
    if (pc->n_large) {
        st = build_large(ctx, pc->bigs_d, pc->n_large, pc->max_Mp, s, &pc->variant);
        if (st != RMB_OK) return cleanup(st);
    }
    int *hf = (int *)(h + hs + hl);
    if (hipMemcpyAsync(hf, pc->flag_d, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup(fail(ctx, RMB_EDEVICE, "preconditioner build failed"));
    if (*hf & 4) return cleanup(fail(ctx, RMB_ENOTSPD, "a body's mobility block is not positive definite"));
    if (*hf & 8) return cleanup(fail(ctx, RMB_ENOTSPD, "a body's K^T M^-1 K block is singular"));
    *out = pc;
    return RMB_OK;
}

rmb_status rmb_precond_factor_shapes(rmb_ctx ctx, const rmb_system *sys, const rmb_shapes *shapes,
                                     const int32_t *body_shape, const double *body_quat, rmb_precond *out,
                                     rmb_stream stream) {
    if (!ctx || !out) return RMB_EINVAL;
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    RMB_TRY(check_system(ctx, sys, true));
    if (!shapes || shapes->n_shapes < 1 || !shapes->shape_off || !shapes->ref_pos)
        return fail(ctx, RMB_EINVAL, "shapes: n_shapes >= 1, shape_off and ref_pos are required");
    if (!body_shape || !body_quat) return fail(ctx, RMB_EINVAL, "body_shape and body_quat are required");
    const int32_t S = shapes->n_shapes;
    const int64_t *so = shapes->shape_off;
    if (so[0] != 0) return fail(ctx, RMB_EINVAL, "shape_off[0] must be 0");
    for (int32_t k = 0; k < S; ++k)
        if (so[k + 1] <= so[k]) return fail(ctx, RMB_EINVAL, "shape %d has no blobs", k);
    const int64_t n_ref = so[S];
    for (int64_t e = 0; e < 3 * n_ref; ++e)
        if (!std::isfinite(shapes->ref_pos[e])) return fail(ctx, RMB_EINVAL, "shape positions must be finite");
    RMB_TRY(check_body_sizes(ctx, so, S));
    const int64_t N = sys->n_bodies;
    for (int64_t p = 0; p < N; ++p) {
        const int32_t k = body_shape[p];
        if (k < 0 || k >= S) return fail(ctx, RMB_EINVAL, "body %lld: shape index %d out of range", (long long)p, k);
        const int64_t nbp = sys->body_off[p + 1] - sys->body_off[p];
        if (nbp != so[k + 1] - so[k])
            return fail(ctx, RMB_EINVAL, "body %lld has %lld blobs, its shape %d has %lld", (long long)p,
                        (long long)nbp, k, (long long)(so[k + 1] - so[k]));
    }

    auto pc = new rmb_precond_s();
    pc->ctx = ctx;
    pc->nb = sys->n_blobs;
    pc->N = N;
    pc->n_shapes = S;
    // device: [factors | ref positions | shape tracking points (0) | shape
    // build items | shape big items | body items | body big items | rotations | flag]
    const size_t fbytes = al(factor_total(so, S) * 8), rbytes = al(n_ref * 24), qbytes = al(S * 24);
    const size_t sib = al(S * sizeof(BodyWork)), sgb = al(S * sizeof(BigBody));
    const size_t ibytes = al(N * sizeof(BodyWork)), gbytes = al(N * sizeof(BigBody)), tbytes = al(N * 72);
    const size_t total = fbytes + rbytes + qbytes + sib + sgb + ibytes + gbytes + tbytes + 256;
    pc->dbuf = (char *)ctx->arena->alloc(total);
    if (!pc->dbuf) {
        delete pc;
        return fail(ctx, RMB_ENOMEM, "shared preconditioner (%zu bytes) exceeds the budget", total);
    }
    char *p0 = pc->dbuf;
    pc->factor = (double *)p0;
    double *ref_d = (double *)(p0 += fbytes);
    double *q0_d = (double *)(p0 += rbytes);
    BodyWork *sitems_d = (BodyWork *)(p0 += qbytes);
    BigBody *sbigs_d = (BigBody *)(p0 += sib);
    pc->items_d = (BodyWork *)(p0 += sgb);
    pc->bigs_d = (BigBody *)(p0 += ibytes);
    pc->rot_d = (double *)(p0 += gbytes);
    pc->flag_d = (int *)(p0 += tbytes);
    auto cleanup = [&](rmb_status st) {
        (void)hipStreamSynchronize(s);
        ctx->arena->free(pc->dbuf);
        delete pc;
        return st;
    };

    // the shapes as a free-space system of S bodies with tracking points at
    // the origin of their reference frames
    rmb_system ref = *sys;
    ref.n_blobs = n_ref;
    ref.n_bodies = S;
    ref.pos = ref_d;
    ref.body_off = so;
    ref.q = q0_d;
    ref.geometry = RMB_GEOM_FREE;
    ref.blob_shift = nullptr;
    BodyLists sl;
    body_items(ref, so, pc->factor, pc->flag_d, sl);
    // per body: the shape's factor, the body's blob range and rotation
    std::vector<int32_t> sidx(S, -1);
    for (size_t i = 0; i < sl.small.size(); ++i) sidx[sl.small[i].body] = (int32_t)i;
    for (size_t i = 0; i < sl.large.size(); ++i) sidx[sl.large[i].w.body] = (int32_t)i;
    std::vector<BodyWork> bs;
    std::vector<BigBody> bl;
    int max_m = 0, max_Mp = 0;
    for (int64_t p = 0; p < N; ++p) {
        const int32_t k = body_shape[p];
        const bool large = is_large_body(so[k + 1] - so[k]);
        BodyWork w = large ? sl.large[sidx[k]].w : sl.small[sidx[k]];
        w.pos = sys->pos;
        w.q = sys->q + 3 * p;
        w.blob0 = sys->body_off[p];
        w.body = (int32_t)p;
        w.wall = 0;
        w.rot = pc->rot_d + 9 * p;
        if (large) {
            BigBody g{};
            g.w = w;
            g.Mp = (int32_t)padded_dim(w.n_blobs);
            bl.push_back(g);
            max_Mp = std::max(max_Mp, g.Mp);
        } else {
            bs.push_back(w);
            max_m = std::max(max_m, 3 * w.n_blobs);
        }
    }
    pc->n_small = (int32_t)bs.size();
    pc->n_large = (int32_t)bl.size();
    pc->max_m = max_m;
    pc->max_Mp = max_Mp;

    const size_t h_ref = n_ref * 24, h_ss = sl.small.size() * sizeof(BodyWork), h_sl = sl.large.size() * sizeof(BigBody);
    const size_t h_bs = bs.size() * sizeof(BodyWork), h_bl = bl.size() * sizeof(BigBody);
    const size_t o_ss = al(h_ref), o_sl = o_ss + al(h_ss), o_bs = o_sl + al(h_sl), o_bl = o_bs + al(h_bs),
                 o_hf = o_bl + al(h_bl);
    char *h = nullptr;
    rmb_status st = pinned(ctx, o_hf + 64, (void **)&h);
    if (st != RMB_OK) return cleanup(st);
    memcpy(h, shapes->ref_pos, h_ref);
    memcpy(h + o_ss, sl.small.data(), h_ss);
    memcpy(h + o_sl, sl.large.data(), h_sl);
    memcpy(h + o_bs, bs.data(), h_bs);
    memcpy(h + o_bl, bl.data(), h_bl);
    if (hipMemsetAsync(pc->flag_d, 0, sizeof(int), s) != hipSuccess ||
        hipMemsetAsync(q0_d, 0, S * 24, s) != hipSuccess ||
        hipMemcpyAsync(ref_d, h, h_ref, hipMemcpyHostToDevice, s) != hipSuccess ||
        (h_ss && hipMemcpyAsync(sitems_d, h + o_ss, h_ss, hipMemcpyHostToDevice, s) != hipSuccess) ||
        (h_sl && hipMemcpyAsync(sbigs_d, h + o_sl, h_sl, hipMemcpyHostToDevice, s) != hipSuccess) ||
        (h_bs && hipMemcpyAsync(pc->items_d, h + o_bs, h_bs, hipMemcpyHostToDevice, s) != hipSuccess) ||
        (h_bl && hipMemcpyAsync(pc->bigs_d, h + o_bl, h_bl, hipMemcpyHostToDevice, s) != hipSuccess) ||
        launch_precond_build_small(sitems_d, (int32_t)sl.small.size(), sl.max_m, s) != hipSuccess ||
        launch_quat_rotations(body_quat, N, pc->rot_d, pc->flag_d, s) != hipSuccess)
        return cleanup(fail(ctx, RMB_EDEVICE, "shared preconditioner build launch failed"));
    if (!sl.large.empty()) {
        int variant = 0;
        st = build_large(ctx, sbigs_d, (int32_t)sl.large.size(), sl.max_Mp, s, &variant);
        if (st != RMB_OK) return cleanup(st);
        pc->variant = variant;
    }
    int *hf = (int *)(h + o_hf);
    if (hipMemcpyAsync(hf, pc->flag_d, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup(fail(ctx, RMB_EDEVICE, "shared preconditioner build failed"));
    if (*hf & 16) return cleanup(fail(ctx, RMB_EINVAL, "a body quaternion is zero or not finite"));
    if (*hf & 4) return cleanup(fail(ctx, RMB_ENOTSPD, "a shape's mobility block is not positive definite"));
    if (*hf & 8) return cleanup(fail(ctx, RMB_ENOTSPD, "a shape's K^T M^-1 K block is singular"));
    *out = pc;
    return RMB_OK;
}

rmb_status rmb_precond_set_orientations(rmb_ctx ctx, rmb_precond pc, const double *body_quat, rmb_stream stream) {
    if (!ctx) return RMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    if (!pc || pc->ctx != ctx) return fail(ctx, RMB_EINVAL, "preconditioner is NULL or from another context");
    if (!pc->rot_d) return fail(ctx, RMB_EINVAL, "preconditioner has no shared shape factors");
    if (!body_quat) return fail(ctx, RMB_EINVAL, "body_quat is required");
    int *hf = nullptr;
    RMB_TRY(pinned(ctx, sizeof(int), (void **)&hf));
    RMB_HIP(ctx, hipMemsetAsync(pc->flag_d, 0, sizeof(int), s));
    RMB_HIP(ctx, launch_quat_rotations(body_quat, pc->N, pc->rot_d, pc->flag_d, s));
    RMB_HIP(ctx, hipMemcpyAsync(hf, pc->flag_d, sizeof(int), hipMemcpyDeviceToHost, s));
    RMB_HIP(ctx, hipStreamSynchronize(s));
    if (*hf & 16) return fail(ctx, RMB_EINVAL, "a body quaternion is zero or not finite");
    return RMB_OK;
}

rmb_status rmb_precond_apply(rmb_ctx ctx, const rmb_precond pc, int32_t nrhs, const double *in, double *out,
                             rmb_stream stream) {
    if (!ctx) return RMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    if (!pc || pc->ctx != ctx) return fail(ctx, RMB_EINVAL, "preconditioner is NULL or from another context");
    if (nrhs < 0 || nrhs > 65535) return fail(ctx, RMB_EINVAL, "nrhs out of range");
    if (nrhs == 0) return RMB_OK;
    if (!in || !out || in == out) return fail(ctx, RMB_EINVAL, "in and out must be distinct device buffers");
    PrecondApplyJob a[2] = {};
    for (int k = 0; k < 2; ++k) {
        a[k].in = in;
        a[k].out = out;
        a[k].ld = 3 * pc->nb + 6 * pc->N;
        a[k].nb3 = 3 * pc->nb;
        a[k].wg_begin = 0;
        a[k].nrhs = nrhs;
    }
    a[0].items = pc->items_d;
    a[0].n_items = pc->n_small;
    a[1].items = (const BodyWork *)pc->bigs_d;
    a[1].n_items = pc->n_large;
    void *d = nullptr, *h = nullptr;
    RMB_TRY(ctx_scratch(ctx, sizeof a, &d));
    RMB_TRY(pinned(ctx, sizeof a, &h));
    memcpy(h, a, sizeof a);
    RMB_HIP(ctx, hipMemcpyAsync(d, h, sizeof a, hipMemcpyHostToDevice, s));
    if (pc->n_small)
        RMB_HIP(ctx, launch_precond_apply_small((const PrecondApplyJob *)d, 1, pc->n_small, nrhs, pc->max_m, s));
    if (pc->n_large)
        RMB_HIP(ctx, launch_precond_apply_large((const PrecondApplyJob *)d + 1, 1, pc->n_large, nrhs, pc->max_Mp, s));
    return RMB_OK;
}

rmb_status rmb_ctx_tuned_panel(rmb_ctx ctx, int32_t padded_dim, int32_t *panel_width) {
    if (!ctx || !panel_width) return RMB_EINVAL;
    auto it = ctx->tuned_panel.find(padded_dim);
    int p = 0, g, c;
    if (it != ctx->tuned_panel.end()) large_variant_shape(it->second, &p, &g, &c);
    *panel_width = p;
    return RMB_OK;
}

int32_t rmb_tile_shape_count(void) { return large_variant_count(); }

rmb_status rmb_tile_shape_info(int32_t shape, int32_t *panel, int32_t *row_tiles, int32_t *chunk) {
    if (shape < 0 || shape >= large_variant_count() || !panel || !row_tiles || !chunk) return RMB_EINVAL;
    int p, g, c;
    large_variant_shape(shape, &p, &g, &c);
    *panel = p, *row_tiles = g, *chunk = c;
    return RMB_OK;
}

rmb_status rmb_ctx_set_tile_shape(rmb_ctx ctx, int32_t padded_dim, int32_t shape) {
    if (!ctx) return RMB_EINVAL;
    if (padded_dim < 64 || padded_dim % 64 || shape < -1 || shape >= large_variant_count())
        return fail(ctx, RMB_EINVAL, "rmb_ctx_set_tile_shape: padded_dim %d, shape %d", padded_dim, shape);
    if (shape < 0) ctx->forced_shape.erase(padded_dim);
    else ctx->forced_shape[padded_dim] = shape;
    return RMB_OK;
}

rmb_status rmb_ctx_tune_log(rmb_ctx ctx, int32_t capacity, rmb_tune_record *records, int32_t *count) {
    if (!ctx || !count || capacity < 0 || (capacity > 0 && !records))
        return ctx ? fail(ctx, RMB_EINVAL, "rmb_ctx_tune_log: bad arguments") : RMB_EINVAL;
    const int32_t total = (int32_t)ctx->tune_log.size();
    for (int32_t i = 0; i < total && i < capacity; ++i) {
        const auto &t = ctx->tune_log[i];
        rmb_tune_record r{};
        r.padded_dim = t.Mp;
        large_variant_shape(t.variant, &r.panel, &r.row_tiles, &r.chunk);
        r.ms = t.ms;
        auto it = ctx->tuned_panel.find(t.Mp);
        r.chosen = it != ctx->tuned_panel.end() && it->second == t.variant;
        records[i] = r;
    }
    *count = total;
    return RMB_OK;
}

void rmb_precond_destroy(rmb_precond pc) {
    if (!pc) return;
    (void)hipDeviceSynchronize();
    pc->ctx->arena->free(pc->dbuf);
    delete pc;
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------

rmb_status rmb_server_create(rmb_ctx ctx, int32_t max_active, rmb_stream stream, rmb_server *out) {
    if (!ctx || !out) return RMB_EINVAL;
    *out = nullptr;
    if (max_active < 0) return fail(ctx, RMB_EINVAL, "max_active must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    auto srv = new rmb_server_s();
    srv->eng = new Engine(ctx, s, max_active ? max_active : 1024);
    rmb_status st = srv->eng->init();
    if (st != RMB_OK) {
        delete srv->eng;
        delete srv;
        return st;
    }
    *out = srv;
    return RMB_OK;
}

rmb_status rmb_server_submit(rmb_server srv, const rmb_system *sys, const double *FT, const double *slip, double *U,
                             double *lambda, const rmb_solve_opts *opts, int64_t tag) {
    if (!srv) return RMB_EINVAL;
    Job *J = nullptr;
    return srv->eng->submit(sys, FT, slip, U, lambda, opts, nullptr, tag, &J);
}

rmb_status rmb_server_step(rmb_server srv, int32_t *n_active, int32_t *n_queued) {
    if (!srv) return RMB_EINVAL;
    Engine *E = srv->eng;
    RMB_TRY(enter(E->ctx, E->s));
    rmb_status st = E->step();
    if (n_active) *n_active = (int32_t)E->active.size();
    if (n_queued) *n_queued = (int32_t)E->queue.size();
    return st;
}

rmb_status rmb_server_poll(rmb_server srv, int32_t max_out, int64_t *tags, rmb_solve_info *infos, int32_t *n_out) {
    if (!srv || !n_out) return RMB_EINVAL;
    Engine *E = srv->eng;
    int32_t n = 0;
    while (n < max_out && !E->done.empty()) {
        Job *J = E->done.front();
        E->done.pop_front();
        if (tags) tags[n] = J->tag;
        if (infos) Engine::fill_info(J, &infos[n]);
        delete J;
        ++n;
    }
    *n_out = n;
    return RMB_OK;
}

void rmb_server_destroy(rmb_server srv) {
    if (!srv) return;
    delete srv->eng;
    delete srv;
}

static rmb_status run_batch(rmb_ctx ctx, int32_t count, const rmb_system *systems, const rmb_precond *pcs,
                            const double *const *FT, const double *const *slip, double *const *U,
                            double *const *lambda, const rmb_solve_opts *opts, rmb_solve_info *infos,
                            hipStream_t s, bool resist = false) {
    Engine E(ctx, s, std::max(1, std::min<int32_t>(count, 1024)));
    RMB_TRY(E.init());
    std::vector<Job *> jobs(count, nullptr);
    for (int32_t i = 0; i < count; ++i) {
        rmb_status st = E.submit(&systems[i], FT[i], slip ? slip[i] : nullptr, U[i], lambda[i], opts,
                                 pcs ? pcs[i] : nullptr, i, &jobs[i], resist);
        if (st != RMB_OK) return st;
    }
    std::vector<rmb_status> status(count, RMB_OK);
    int32_t left = count;
    while (left > 0) {
        RMB_TRY(E.step());
        while (!E.done.empty()) {
            Job *J = E.done.front();
            E.done.pop_front();
            if (infos) Engine::fill_info(J, &infos[J->tag]);
            status[J->tag] = J->status;
            if (J->status != RMB_OK && !J->msg.empty()) ctx->err = J->msg;
            delete J;
            --left;
        }
    }
    for (int32_t i = 0; i < count; ++i)
        if (status[i] != RMB_OK) return status[i];
    return RMB_OK;
}

rmb_status rmb_solve_mobility(rmb_ctx ctx, const rmb_system *sys, const rmb_precond pc, const double *FT,
                              const double *slip, double *U, double *lambda, const rmb_solve_opts *opts,
                              rmb_solve_info *info, rmb_stream stream) {
    if (!ctx) return RMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    rmb_solve_info tmp{};
    rmb_precond pcs[1] = {pc};
    const double *slips[1] = {slip};
    return run_batch(ctx, 1, sys, pc ? pcs : nullptr, &FT, slips, &U, &lambda, opts, info ? info : &tmp, s);
}

rmb_status rmb_solve_resistance(rmb_ctx ctx, const rmb_system *sys, const rmb_precond pc, const double *U,
                                const double *slip, double *F, double *lambda, const rmb_solve_opts *opts,
                                rmb_solve_info *info, rmb_stream stream) {
    if (!ctx) return RMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    rmb_solve_info tmp{};
    rmb_precond pcs[1] = {pc};
    const double *slips[1] = {slip};
    return run_batch(ctx, 1, sys, pc ? pcs : nullptr, &U, slips, &F, &lambda, opts, info ? info : &tmp, s, true);
}

rmb_status rmb_solve_batch(rmb_ctx ctx, int32_t count, const rmb_system *systems, const double *const *FT,
                           const double *const *slip, double *const *U, double *const *lambda,
                           const rmb_solve_opts *opts, rmb_solve_info *infos, rmb_stream stream) {
    if (!ctx) return RMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    RMB_TRY(enter(ctx, s));
    if (count < 0 || !systems || !FT || !U || !lambda || !infos)
        return fail(ctx, RMB_EINVAL, "bad batch arguments");
    if (count == 0) return RMB_OK;
    return run_batch(ctx, count, systems, nullptr, FT, slip, U, lambda, opts, infos, s);
}

}  // extern "C"

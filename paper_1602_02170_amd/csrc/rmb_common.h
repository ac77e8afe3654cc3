// Shared declarations of the rigid-multiblob GPU library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rmb.h"

namespace rmb {

// Device pointers read from job tables are generic to the compiler, so their
// loads become flat loads, which count against both the vector-memory and the
// LDS counters and force full waits.  A global-address-space view gives
// global loads that the compiler can wait on one at a time.
template <typename T>
using gmem = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gmem<T> as_global(T *p) {
    return (gmem<T>)p;
}


// ---------------------------------------------------------------------------
// pair-product work description
// ---------------------------------------------------------------------------

// Source record of the FP32-pair product: position in FP64 (the difference
// r_i - r_j is formed in FP64 and rounded once), force and height in FP32.
struct alignas(8) SrcF32 {
    double x, y, z;
    float fx, fy, fz, zf;
};

// Source record of the FP64 product.
struct alignas(16) SrcF64 {
    double x, y, z, fx, fy, fz;
};

constexpr int kPairBlock = 256;  // targets per workgroup (4 waves of 64)
constexpr int kAccBlock = 64;    // FP32 sums are flushed to FP64 every 64 sources

// One system's share of a pair-product launch.  Workgroups
// [tile_begin, tile_begin + n_tblock * n_split) of the launch belong to it;
// local workgroup w covers targets [(w % n_tblock) * 256, +256) against
// sources [(w / n_tblock) * chunk, +chunk) and writes partial slot
// w / n_tblock.
struct PairJob {
    const double *tpos;  // [nb][3] target positions
    const void *src;     // [ns] SrcF32 or SrcF64 records
    double *partial;     // [n_split][nb][3] per-split sums (no prefactor)
    int64_t nb;          // targets
    int64_t ns;          // sources (= nb for the mobility product)
    int64_t tile_begin;
    int64_t chunk;
    int32_t n_tblock;
    int32_t n_split;
    // RPY constants (eq:RPYTensor): a, 4a^2, 9/(32a), 3/(32a) (the FP32
    // kernel takes lengths in units of a and uses a alone)
    double a, four_a2, k_near_iso, k_near_rr;
};

hipError_t launch_store_pair_job(const PairJob &j, PairJob *dst, hipStream_t s);

// Number of source splits and the split length for a system of nb blobs.
// A function of nb only, so that a system's arithmetic does not depend on
// what else shares the launch.
void split_plan(int64_t nb, int32_t *n_split, int64_t *chunk, int32_t *n_tblock);

// The same for nt targets and ns sources.
void split_plan_rect(int64_t nt, int64_t ns, int32_t *n_split, int64_t *chunk, int32_t *n_tblock);

// Fills the plan fields and constants of a PairJob (targets = sources).
void pair_job_init(PairJob *J, const double *tpos, const void *src, double *partial, int64_t nb,
                   double a);
// Rectangular product: nt target positions, ns source records, radius a.
void pair_job_init_rect(PairJob *J, const double *tpos, int64_t nt, const void *src, int64_t ns, double *partial,
                        double a);
// Sources for a flow field: record i * n_sub + k is blob i moved by a * off[k]
// (off: device [n_sub][3]) carrying lambda_i / n_sub; flag |= 1 for a
// non-finite position, 2 for z <= 0 when `wall`.
hipError_t launch_pack_sub_sources(int precision, const double *pos, const double *lam, int64_t nb, const double *off,
                                   int32_t n_sub, double a, int wall, void *src, int *flag, hipStream_t s);

// One system's share of a launch of the pair kernel that evaluates each pair
// block once (pair_sym_kernel).  The T(T+1)/2 block pairs (I <= J) of its
// T = ceil(nb / B) blocks are numbered row by row; they are evaluated in
// bands of whole rows [I0, I1) (tiles [t0, t0 + band tiles)), so that the
// partial sums of one band at a time are stored: workgroups [wg_begin,
// wg_begin + band tiles) are the band's tiles, and reduction workgroups
// [red_begin, red_begin + sym_reduce_groups_band(...)) add the band's
// partials of every blob they touch into an FP64 accumulator (first band:
// stored; later bands: added), the last band writing the result.
struct SymJob {
    const double *tpos;  // [nb][3] positions
    const double *lam;   // [nb][3] operand (the target's own force for M^T lambda)
    double *vpart;       // [band tiles][3][B] target-side sums (FP32 pairs with B = 64: floats at the same base)
    double *upart;       // [band tiles][3][B] source-side sums (likewise)
    double *vel;         // [nb][3] result, prefactor applied (unused with epi)
    double *acc;         // [nb][3] FP64 sums of the bands so far (several bands only; may be vel)
    const void *epi;     // NULL, or the system's saddle-operator rows (a SaddleJob): the
                         // reduction then writes the blob rows of A x (or b - A x) instead of vel
    int64_t nb;
    int64_t wg_begin;
    int64_t red_begin;
    int64_t t0;          // first tile of the band
    int32_t n_blk;
    int32_t B;
    int32_t I0, I1;      // block rows of the band
    int32_t first, last; // the band is the system's first / last
    int32_t f32;         // FP32 pairs (with B = 64 the tile partials are floats)
    int32_t pad;
    double a;            // blob radius (the kernel takes lengths in units of a)
    double pref;
};

// Block size and block count of the symmetric product for nb blobs (a
// function of nb only); tiles it evaluates.
void sym_plan(int64_t nb, int32_t *B, int32_t *n_blk);
int64_t sym_tiles(int64_t nb);
// Bands: consecutive block rows whose tiles' partials (counted in FP64,
// whatever the pair precision, so that the partition depends on nb alone)
// fit `band_bytes`; a single row always forms a band of its own.
struct SymBand {
    int32_t I0, I1;
    int64_t t0, tiles;
};
// Default partial storage of one band: 4 GiB, so that every product up to
// about 210,000 blobs runs in one band and larger ones in a few.
constexpr size_t kSymBandBytes = size_t(4) << 30;
std::vector<SymBand> sym_bands(int64_t nb, size_t band_bytes);
// Doubles of partial storage for the largest band (vpart + upart).
size_t sym_band_partial_doubles(int64_t nb, size_t band_bytes);
// Reduction workgroups of one band: blobs of blocks [I0, T), or all blobs
// for the last band (which writes every blob's result).
int64_t sym_reduce_groups_band(int64_t nb, int32_t B, const SymBand &b, bool last);
// One job record written to device memory by a kernel (from its argument).
hipError_t launch_store_sym_job(const SymJob &j, SymJob *dst, hipStream_t s);
// Systems of at least this many blobs use the symmetric product.
constexpr int64_t kSymMinBlobs = 1024;
inline bool use_sym(int64_t nb) { return nb >= kSymMinBlobs; }
hipError_t launch_pair_sym(int precision, bool wall, int B, const SymJob *jobs, int32_t n_jobs, int64_t n_tiles,
                           hipStream_t s);
// n_wg reduction workgroups (sym_reduce_groups_band per job), then
// (n_body + 15) / 16 more for the saddle body rows of `sd` (none when sd is
// null).
struct SaddleJob;
hipError_t launch_sym_reduce(const SymJob *jobs, int32_t n_jobs, int64_t n_wg, const SaddleJob *sd, int32_t n_sd,
                             int64_t n_body, hipStream_t s);

// Packing of source records for several systems in one launch.
struct PackJob {
    const double *pos;
    const double *lam;  // lambda part of the operand (first 3 nb entries)
    void *src;
    int64_t nb;
    int64_t wg_begin;   // first 256-blob workgroup of this system
    int32_t precision;
    int32_t pad;
};

// Kernel launchers (rmb_pair.hip).
hipError_t launch_pack_table(const PackJob *jobs, int32_t n_jobs, int64_t n_wg, hipStream_t s);
hipError_t launch_pack_sources(int precision, const double *pos, const double *lam, int64_t nb,
                               void *src, hipStream_t s);
// jobs: device array of n_jobs PairJob with increasing tile_begin; n_tiles is
// the total workgroup count.
// FP32 one-sided product with LDS-staged sources (same jobs and partials as
// the FP32 case of launch_pair_tiles, which uses it)
hipError_t launch_pair_lds_f32(bool wall, const PairJob *jobs, int32_t n_jobs, int64_t n_tiles, hipStream_t s);
hipError_t launch_pair_tiles(int precision, bool wall, const PairJob *jobs, int32_t n_jobs,
                             int64_t n_tiles, hipStream_t s);
// v[i] = pref * sum_s partial[s][i]
hipError_t launch_reduce_partials(const double *partial, int32_t n_split, int64_t nb, double pref,
                                  double *v, hipStream_t s);
// flag |= 1 for a non-finite coordinate, |= 2 for z <= 0 when wall != 0,
// |= 32 for a permeability shift (if given) that is negative or not finite
hipError_t launch_validate_positions(const double *pos, int64_t nb, int wall, const double *shift, int *flag,
                                     hipStream_t s);
// v_i += shift_i lambda_i for every blob (no-op when shift is NULL)
hipError_t launch_add_shift(const double *shift, const double *lam, int64_t nb, double *v, hipStream_t s);

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------

// First-fit sub-allocator over large hipMalloc blocks, capped at a budget.
class Arena {
  public:
    explicit Arena(size_t budget) : budget_(budget) {}
    ~Arena();
    // Returns nullptr when the budget would be exceeded or hipMalloc fails.
    void *alloc(size_t bytes);
    void free(void *p);
    size_t budget() const { return budget_; }
    size_t in_use() const { return in_use_; }
    // Returns blocks with no live allocation to HIP.
    void release_free_blocks();

  private:
    struct Seg {
        size_t off, size;
        bool used;
    };
    struct Block {
        char *base;
        size_t size;
        std::vector<Seg> segs;
    };
    std::vector<Block> blocks_;
    size_t budget_;
    size_t reserved_ = 0;
    size_t in_use_ = 0;
};

}  // namespace rmb

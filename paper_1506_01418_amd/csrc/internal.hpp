// Internal types shared by the host runtime and the kernels of libpsgld.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "model.hpp"
#include "psgld.h"

namespace psgld {

// One training entry as the sparse kernel streams it (8 bytes): the offset
// of the partner row/column in its factor array (index * Kp) and the value.
struct Entry {
    int32_t off;
    float val;
};

// Floats per stored factor row: K padded so rows never straddle 128-byte
// cache lines more than they must -- a power of two (at least 4) up to 32,
// else a multiple of 32.  The padding is held at zero.
inline int padded_rank(int K)
{
    if (K > 32) return (K + 31) / 32 * 32;
    int p = 4;
    while (p < K) p *= 2;
    return p;
}

// Entries past the end of every entry array, so a batch of reads that
// starts inside an item never leaves the allocation.
constexpr int kEntryPad = 16;
// Floats past the end of every factor array: a group's lanes beyond ceil(K/4)
// read (and discard) up to one row past the row they address.
constexpr int kFactorPad = 256;

// One held-out cell attached to a row: partner column offset (col * Kp)
// and output slot.
struct HeldEntry {
    int32_t off;
    int32_t slot;
};

// Work of one work-group within one part.  side 0 = rows of W, 1 = columns
// of H.  Each of its Q groups handles the item of its GroupRec; items are
// split over G = 2^glog2 consecutive groups.  n_split > 0 marks one share of
// an item split over n_split work-groups: shares write partial gradients to
// scratch slots split_first .. split_first + n_split - 1 and the last share
// to finish combines them in slot order and applies the update.
struct WgTask {
    int16_t side;
    int16_t glog2;
    int32_t split_first;
    int32_t split_idx;   // 32-bit: an item of up to 2^31 entries may be cut into that many shares
    int32_t n_split;
};
static_assert(sizeof(WgTask) == 16, "a work-group task is 16 bytes");

// One group's item (-1 = none) and its range of entries [s0, s1).
struct GroupRec {
    int32_t item;
    int32_t s0;
    int32_t s1;
    int32_t lead;   // 1 if this group applies the item's update
};


// Which global iteration a launch runs, and the scalars that depend on it.
// Step sizes are computed on the host in FP64 (eps_t = a (t0 + t)^-gamma and
// sqrt(2 eps_t), each rounded once to FP32) into a device table indexed by t;
// a launch finds t as *clock + k, so a captured sequence of launches replays
// for any starting iteration once the host has set the clock.
struct IterClock {
    const float2 *eps_tab;    // (eps_t, sigma_t) for t = 0 .. table length - 1
    const int32_t *clock;     // device iteration counter, or null (t = k)
    int32_t k;
    int32_t burn_in, thin;    // moments at t >= burn_in with (t - burn_in) % thin == 0
    int32_t bookkeeping;      // 0: no moments and no held-out sums (tuning trials)
    int32_t has_heldout;
};

struct IterScalars {
    uint32_t t;
    float eps, sigma;
    bool do_moments, do_heldout;
};

__device__ __forceinline__ IterScalars iter_scalars_at(int32_t t, const float2 *eps_tab, int32_t burn_in,
                                                     int32_t thin, bool bookkeeping, bool has_heldout)
{
    IterScalars s;
    const float2 es = eps_tab[t];
    s.t = static_cast<uint32_t>(t);
    s.eps = es.x;
    s.sigma = es.y;
    const bool post = bookkeeping && t >= burn_in;
    s.do_moments = post && (t - burn_in) % thin == 0;
    s.do_heldout = post && has_heldout;
    return s;
}

__device__ __forceinline__ IterScalars iter_scalars(const IterClock &c)
{
    const int32_t t = (c.clock ? *c.clock : 0) + c.k;
    return iter_scalars_at(t, c.eps_tab, c.burn_in, c.thin, c.bookkeeping != 0, c.has_heldout != 0);
}

// Arguments of one sparse iteration (one part), passed by value.
struct SparseIterArgs {
    const float *x_old[2];   // [0] W (I x Kp), [1] H stored J x Kp
    float *x_new[2];
    const int32_t *ptr[2];   // part's row / column offsets into ent[side] (length I+1 / J+1)
    const Entry *ent[2];     // row-sorted (partner = column) / column-sorted (partner = row)
    const WgTask *tasks;     // part's work-group tasks, in dispatch order
    const GroupRec *recs;    // part's group records: Q per task
    int32_t n_tasks;
    float *split_partial;    // scratch: Kp floats per split share
    int32_t *split_count;    // arrival counters, one per split item (kept at 0 between launches)
    int32_t K, Kp, nq;
    float scale;             // s_p = N / |part p|
    float lambda[2];
    float inv_phi, beta, mu_floor;
    uint32_t seed_lo, seed_hi;
    int32_t mirror, prior_kind;
    uint32_t flags;          // PSGLD_TEST_* bits
    IterClock clk;
    double *sum[2], *sum2[2];
    const int32_t *ho_ptr;   // part's held-out row offsets (length I+1)
    const HeldEntry *ho_ent;
    double *ho_sum;
    int32_t *nonfinite;      // min iteration with a non-finite result
};

// A context as the batched kernel sees it: everything that stays fixed
// between iterations, in device memory.  The iteration t comes from the
// context's own clock; the part is t mod B, the buffer read is
// (t + cur_phase) & 1, and the part's tables are indexed by the part.
struct JobDesc {
    float *W[2], *H[2];
    const int32_t *rowptr, *colptr;   // part-major: B x I and B x J offsets (+1)
    const Entry *ent[2];
    const WgTask *tasks;
    const GroupRec *recs;
    const int32_t *task_off;          // per part: its first task
    const int32_t *n_tasks;           // per part
    const float *scale;               // per part: s_p
    float *split_partial;
    int32_t *split_count;
    int32_t I, J, K, Kp, nq, B;
    float lambda[2];
    float inv_phi, beta, mu_floor;
    uint32_t seed_lo, seed_hi;
    int32_t mirror, prior_kind;
    uint32_t flags;
    const float2 *eps_tab;            // indexed by the global iteration
    const int32_t *part_tab;          // part of each global iteration, or null (t mod B)
    const int32_t *clock;
    int32_t cur_phase;
    int32_t burn_in, thin, has_heldout;
    double *sum[2], *sum2[2];
    const int32_t *ho_ptr;            // part-major, B x I (+1), or null
    const HeldEntry *ho_ent;
    double *ho_sum;
    int32_t *nonfinite;
};

// One batched launch: up to kMaxBatch contexts of one kernel variant;
// work-groups [wg_first[j], wg_first[j + 1]) serve context j (its largest
// part's task count; work-groups past the current part's count exit).
constexpr int kMaxBatch = 64;
struct BatchArgs {
    const JobDesc *jobs[kMaxBatch];
    int32_t wg_first[kMaxBatch + 1];
    int32_t n;
    int32_t k;   // this launch runs iteration *clock + k of every context
};

hipError_t launch_sparse_batch(const BatchArgs &b, int lik, int lanes_per_group, int quads_per_lane,
                               hipStream_t stream);
// *clocks[j] += delta[j] for j < n.
hipError_t launch_advance_clocks(int32_t *const *clocks, const int32_t *delta, int n, hipStream_t stream);
// n_iter iterations of the batch in one cooperative launch of `grid`
// work-groups (<= 0: as many as the device holds at once, capped by the
// work), with `barrier` (one device word, reset by the launch) as the
// grid-wide barrier counter; the clocks are not advanced.
hipError_t launch_sparse_persistent(const BatchArgs &b, int n_iter, int lik, int lanes_per_group, int quads_per_lane,
                                    int grid, uint32_t *barrier, hipStream_t stream);

// Launches one sparse iteration with the kernel variant chosen for (K, lik).
hipError_t launch_sparse_iter(const SparseIterArgs &a, int lik, int lanes_per_group, int quads_per_lane,
                              hipStream_t stream);
int sparse_threads_per_group(int K);
int sparse_quads_per_lane(int K);
int sparse_lanes_for(int K, int qpl);
bool sparse_variant_exists(int lpg, int qpl);
int sparse_block_threads();

// Tunable shape of the sparse schedule (chosen per context by psgld_tune).
struct ScheduleParams {
    int entries_per_group = 64;   // entries a group takes before an item gets more groups
    bool split_items = true;      // cut items longer than a work-group's share over several work-groups
    bool xcd_remap = true;        // place each block's work on one XCD
};


// Host-side schedule of one part: work-group tasks and group records.
struct PartSchedule {
    std::vector<WgTask> tasks;
    std::vector<GroupRec> recs;
    int32_t n_splits = 0;   // scratch slots used
};
// pre: offsets of the part's entries per row (length I+1) and per column
// (length J+1); pieces of rows / columns; the part index p; skip_block[b]
// (may be NULL) marks part blocks b handled elsewhere (dense blocks).
void build_part_schedule(const int32_t *pre_r, const int32_t *pre_c, int64_t I, int64_t J,
                         const std::vector<int32_t> &row_piece, const std::vector<int32_t> &col_piece,
                         int32_t B, int32_t p, int lanes_per_group, const ScheduleParams &prm,
                         const uint8_t *skip_block, PartSchedule &out);

// ---- dense blocks --------------------------------------------------------
constexpr int kDenseTileCols = 64;   // columns of one MFMA sub-tile
constexpr int kDenseSubTiles = 4;    // sub-tiles (consecutive) per work-group
constexpr int kDenseMaxRows = 128;   // dense blocks have at most this many rows
constexpr int kDenseMaxK = 64;       // and rank at most this

// A dense block of a part: rows [row0, row0 + m), columns [col0, col0 + n);
// its values are stored row-major at v_off with row stride ld = n rounded up
// to kDenseRowAlign cells (padding cells hold 0), so every row starts on a
// 64-byte boundary.  Every stored cell also has a 2-bit code (0 missing, 1
// training, 2 held-out) in an array parallel to the values, 16 cells per
// 32-bit word: cell c is bits 2 (c mod 16) of word c / 16.  Each of its
// n_tiles work-groups takes n_sub consecutive 64-column sub-tiles (fewer for
// taller blocks, so every work-group has about the same work); their W
// partials occupy slots first_partial .. + n_tiles.
constexpr int kDenseRowAlign = 16;
struct DenseBlock {
    int32_t row0, m, col0, n;
    int64_t v_off;
    int32_t first_partial, n_tiles;
    int32_t ld, n_sub;
};

// Code of stored cell c of the dense blocks: 0 missing, 1 training, 2 held-out.
__host__ __device__ __forceinline__ uint32_t dense_code(const uint32_t *codes, int64_t c)
{
    return (codes[c >> 4] >> (2 * (c & 15))) & 3u;
}

// One work-group's share of a block: columns [col, col + n_sub * 64)
// of part block `block`; its W partial goes to slot `partial`; the held-out
// cells of its sub-tile s are heldout[ho[s] .. ho[s + 1]).
struct DenseTile {
    int32_t block;
    int32_t col;
    int32_t partial;
    int32_t ho[kDenseSubTiles + 1];
};

// Dense-block cell codes: 0 missing, 1 training cell, 2 held-out cell.
constexpr uint8_t kMaskTrain = 1;
constexpr uint8_t kMaskHeld = 2;

// A held-out cell inside a dense block, listed with the work-group that
// covers it: row in the block, column relative to the work-group's first
// column, and output slot.
struct DenseHeld {
    int32_t row, col, slot, pad;
};

struct DenseIterArgs {
    const float *x_old[2];
    float *x_new[2];
    const DenseBlock *blocks;   // the part's dense blocks
    int32_t n_blocks;
    const DenseTile *tiles;     // the part's tiles
    int32_t n_tiles;
    const float *val;           // FP32 values, or
    const uint16_t *val16;      // BF16 values (the other pointer is null)
    const uint32_t *mask;       // 2-bit cell codes
    float *w_partial;           // slot_rows x Kp floats per tile
    int32_t slot_rows;          // rows of every W partial slot (the largest padded block height)
    int32_t row_align;          // block heights are padded to this (16 FP32, 32 BF16)
    int32_t K, Kp, KS;          // KS = K rounded up to row_align
    float scale;
    float lambda[2];
    float inv_phi, beta, mu_floor;
    uint32_t seed_lo, seed_hi;
    int32_t mirror, prior_kind;
    uint32_t flags;
    IterClock clk;              // has_heldout: dense blocks hold held-out cells
    double *sum[2], *sum2[2];
    const DenseHeld *heldout;   // held-out cells of dense blocks, grouped by tile
    double *ho_sum;
    int32_t *nonfinite;
};

// Enqueues the dense work of one iteration (tiles with their held-out
// sums, then the W rows).
hipError_t launch_dense_iter(const DenseIterArgs &a, int lik, bool bf16, int max_m, hipStream_t stream);
// A value stored in BF16, widened exactly.
__host__ __device__ inline float bf16_value(uint16_t b)
{
    uint32_t u = static_cast<uint32_t>(b) << 16;
    float f;
    __builtin_memcpy(&f, &u, sizeof f);
    return f;
}
// Raises the dynamic LDS limit of the tile kernels for blocks of max_m rows.
hipError_t dense_prepare(int max_m, int KS);
size_t dense_lds_bytes(int max_m, int KS);
// FP64 log-likelihood partials of all dense blocks' training cells (values
// in val, or in BF16 in val16 when val is null).
hipError_t launch_dense_loglik(const float *W, const float *Hs, const DenseBlock *blocks, int n_blocks,
                               const float *val, const uint16_t *val16, const uint32_t *mask, int K, int Kp,
                               double beta, double phi, double mu_floor, double *partials, int per_block,
                               hipStream_t stream);

hipError_t launch_philox_blocks(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out,
                                hipStream_t stream);
hipError_t launch_normals(int64_t n, uint64_t seed, const int64_t *t, const uint32_t *stream_id,
                          const int64_t *index, int K, float *z, float *radius, hipStream_t stream);
// FP64 training log-likelihood partials over all parts' row-sorted entries
// (n_blocks partials), then an in-order sum of n partials into *out.
hipError_t launch_loglik(const float *W, const float *Hs, const int32_t *row_of_entry,
                         const Entry *ent, int64_t n, int K, int Kp, double beta, double phi,
                         double mu_floor, double *partials, int n_blocks, hipStream_t stream);
hipError_t launch_sum_in_order(const double *partials, int n, double *out, hipStream_t stream);
// *clock = value, and *clock += delta, as kernels (so both can be captured).
hipError_t launch_set_clock(int32_t *clock, int32_t value, hipStream_t stream);
hipError_t launch_advance_clock(int32_t *clock, int32_t delta, hipStream_t stream);
// p[0 .. n) = value, as a kernel (no memset node when captured).
hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t n, hipStream_t stream);

}  // namespace psgld

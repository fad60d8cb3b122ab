// Internal types shared by the host runtime and the kernels of libpsgld.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "psgld.h"

namespace psgld {

// One training entry as the sparse kernel streams it (8 bytes): the offset
// of the partner row/column in its factor array (index * Kp) and the value.
struct Entry {
    int32_t off;
    float val;
};

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
    int32_t side;
    int32_t glog2;
    int32_t split_first;
    int16_t split_idx;
    int16_t n_split;
};

// One group's item (-1 = none) and its range of entries [s0, s1).
struct GroupRec {
    int32_t item;
    int32_t s0;
    int32_t s1;
    int32_t lead;   // 1 if this group applies the item's update
};

enum Lik : int { LIK_GAUSS = 0, LIK_POISSON = 1, LIK_GENERAL = 2 };

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
    float eps, sigma, scale;
    float lambda[2];
    float inv_phi, beta, mu_floor;
    uint32_t seed_lo, seed_hi, t;
    int32_t mirror, prior_kind;
    uint32_t flags;          // PSGLD_TEST_* bits
    int32_t do_moments;
    double *sum[2], *sum2[2];
    int32_t do_heldout;
    const int32_t *ho_ptr;   // part's held-out row offsets (length I+1)
    const HeldEntry *ho_ent;
    double *ho_sum;
    int32_t *nonfinite;      // min iteration with a non-finite result
};

// Launches one sparse iteration with the kernel variant chosen for (K, lik).
hipError_t launch_sparse_iter(const SparseIterArgs &a, int lik, int lanes_per_group,
                              hipStream_t stream);
int sparse_threads_per_group(int K);
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
// (length J+1); pieces of rows / columns; the part index p.
void build_part_schedule(const int32_t *pre_r, const int32_t *pre_c, int64_t I, int64_t J,
                         const std::vector<int32_t> &row_piece, const std::vector<int32_t> &col_piece,
                         int32_t B, int32_t p, int lanes_per_group, const ScheduleParams &prm,
                         PartSchedule &out);

hipError_t launch_philox_blocks(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out,
                                hipStream_t stream);
hipError_t launch_normals(int64_t n, uint64_t seed, const int64_t *t, const uint32_t *stream_id,
                          const int64_t *index, int K, float *z, float *radius, hipStream_t stream);
// FP64 training log-likelihood over all parts' row-sorted entries.
hipError_t launch_loglik(const float *W, const float *Hs, const int32_t *row_of_entry,
                         const Entry *ent, int64_t n, int K, int Kp, double beta, double phi,
                         double mu_floor, double *partials, int n_blocks, double *out,
                         hipStream_t stream);

}  // namespace psgld

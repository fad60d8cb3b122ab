// Internal types shared by the host runtime and the kernels of libpsgld.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "psgld.h"

namespace psgld {

// One training entry as the sparse kernel streams it: the index of the
// partner row/column and the value (8 bytes).
struct Entry {
    int32_t idx;
    float val;
};

// One held-out cell attached to a row: partner column and output slot.
struct HeldEntry {
    int32_t col;
    int32_t slot;
};

// A work-group's share of one part: `count` consecutive items of the part's
// size-sorted item list starting at `first`, each handled by G groups.
// side 0 = rows of W, 1 = columns of H.
struct Task {
    int32_t side;
    int32_t first;
    int32_t count;
    int32_t G;
};

enum Lik : int { LIK_GAUSS = 0, LIK_POISSON = 1, LIK_GENERAL = 2 };

// Arguments of one sparse iteration (one part), passed by value.
struct SparseIterArgs {
    const float *x_old[2];   // [0] W (I x Kp), [1] H stored J x Kp
    float *x_new[2];
    const int32_t *ptr[2];   // part's row / column offsets into ent[side] (length I+1 / J+1)
    const Entry *ent[2];     // row-sorted (partner = column) / column-sorted (partner = row)
    const int32_t *items;    // part's item list: rows sorted, then columns sorted
    const Task *tasks;       // part's tasks
    int32_t n_tasks;
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

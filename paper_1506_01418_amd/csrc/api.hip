// Host runtime of libpsgld: the C ABI declared in psgld.h.
//
// Layout in device memory (HBM), built once on the host at load time:
//  * W is I x Kp and H is stored transposed, J x Kp (Kp = padded_rank(K):
//    rows padded to whole cache lines, padding held at zero), each twice
//    (ping-pong): an
//    iteration reads one copy and writes the other, so every row and column
//    update reads only the previous state (Eq. (8)-(9)).
//  * Training entries are bucketed by part (part of (i,j) = (c - b) mod B
//    for row piece b and column piece c) and stored twice, part-major:
//    row-sorted for the W items (partner = column) and column-sorted for the
//    H items (partner = row).  Offsets are prefix sums over (part, row) and
//    (part, column), so part p's row offsets are a contiguous slice.
//  * For every part, a work schedule: work-group tasks and per-group item
//    records (built in schedule.hip).
//  * FP64 running sums of x and x^2, and FP64 held-out predictive sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"
#include "runtime.hpp"
#include "noise.hpp"
#include "psgld.h"

using namespace psgld;

namespace {

thread_local std::string g_create_error;
constexpr uint32_t kStateMagic = 0x50534744u;  // "PSGD"
constexpr uint32_t kStateVersion = 1;
constexpr int kDenseLLPerBlock = 16;   // work-groups per dense block in the log-likelihood
// Training entries held as coordinates: the kernels index the entry arrays
// with 32-bit integers, up to a batch and the padding past the last entry.
constexpr int64_t kMaxEntries = INT32_MAX - 64;

bool is_gfx950(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return false;
    return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

}  // namespace

struct psgld_ctx {
    int64_t I = 0, J = 0;
    int32_t K = 0, B = 0, Kp = 0, nq = 0, lpg = 0, qpl = 1;
    psgld_likelihood lik{};
    psgld_prior prior{};
    psgld_options opt{};
    int lik_kind = LIK_GENERAL;
    std::string err;

    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool device_ready = false;
    bool loaded = false, factors_set = false, heldout_loaded = false;

    std::vector<int32_t> row_piece, col_piece;
    std::vector<int32_t> pre_r, pre_c;   // entry offsets per (part, row) and (part, column)
    ScheduleParams sched;
    int64_t N = 0;
    std::vector<int64_t> n_p;
    std::vector<int64_t> task_off, n_tasks;
    int32_t max_splits = 0;           // split-share slots the largest part needs

    std::map<void *, size_t> allocs;   // device blocks of the context and their sizes
    int64_t bytes = 0;
    float *W[2] = {nullptr, nullptr}, *H[2] = {nullptr, nullptr};
    int cur = 0;
    int32_t *rowptr = nullptr, *colptr = nullptr;
    Entry *ent_r = nullptr, *ent_c = nullptr;
    int32_t *row_of_entry = nullptr;
    WgTask *tasks = nullptr;
    GroupRec *recs = nullptr;
    float *split_partial = nullptr;
    int32_t *split_count = nullptr;
    double *sum[2] = {nullptr, nullptr}, *sum2[2] = {nullptr, nullptr};
    int64_t n_kept = 0;

    int64_t n_ho = 0;
    int32_t *ho_ptr = nullptr;
    HeldEntry *ho_ent = nullptr;
    double *ho_sum = nullptr;
    std::vector<float> ho_val;
    bool ho_has_val = false;
    std::vector<int32_t> ho_part;
    std::vector<int32_t> ho_slot;           // caller's held-out index -> position of its FP64 sum
    std::vector<int64_t> part_visits;

    // dense blocks (psgld_load_dense)
    int64_t nnz_sparse = 0;                 // training entries stored as coordinates
    std::vector<uint8_t> skip;              // skip[p * B + b]: block (b, (b+p) mod B) is dense
    std::vector<int32_t> dblock_of;         // (b * B + c) -> index into dblocks_host, or -1
    std::vector<DenseBlock> dblocks_host;   // part-major
    std::vector<DenseTile> dtiles_host;     // part-major, a block's work-groups consecutive
    std::vector<int64_t> dblock_first_tile; // index into dtiles_host of each block's first work-group
    std::vector<int64_t> dblk_off, dblk_cnt, dtile_off, dtile_cnt;
    std::vector<uint8_t> dmask_host;
    DenseBlock *dblocks = nullptr;
    DenseTile *dtiles = nullptr;
    float *dval = nullptr;
    uint16_t *dval16 = nullptr;             // the values in BF16 (PSGLD_BF16_DENSE_VALUES; dval is then null)
    uint32_t *dmask = nullptr;              // 2-bit cell codes of the dense blocks
    std::vector<uint32_t> dcodes_host;      // their host copy
    float *w_partial = nullptr;
    DenseHeld *dheld = nullptr;
    int dense_max_m = 0, KS = 0;

    int32_t *nonfinite = nullptr;
    double *ll_partials = nullptr, *ll_out = nullptr;
    int ll_blocks = 0;
    int64_t t = 0;

    // step sizes (eps_t, sigma_t) for t in [eps_base, eps_base + eps_cap)
    float2 *eps_tab = nullptr;
    int32_t *part_tab = nullptr;      // part of each iteration of the window (random order only)
    int64_t eps_base = 0, eps_cap = 0;
    psgld_eps_schedule eps_sched{};
    // device iteration counter read by captured graphs; clock_host is its
    // value once the enqueued work has run (-1: not set yet)
    int32_t *clock = nullptr;
    uint32_t *barrier = nullptr;      // grid-wide barrier counter of persistent launches
    int64_t clock_host = -1;
    hipStream_t cap_stream = nullptr;
    // captured runs of iterations, by (first part, ping-pong buffer, length)
    std::map<std::tuple<int32_t, int32_t, int64_t>, hipGraphExec_t> graphs;
    // batched stepping: per-part tables and the context's job description
    int32_t *task_off_dev = nullptr, *n_tasks_dev = nullptr;
    float *scale_dev = nullptr;
    int32_t max_tasks = 0;
    JobDesc *job_desc = nullptr;
    JobDesc job_host{};
    bool job_valid = false;

    psgld_status fail(psgld_status s, const std::string &msg)
    {
        err = msg;
        return s;
    }
};

#define HIPTRY(ctx, expr)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return (ctx)->fail(PSGLD_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Makes `dev` the calling thread's device; hipSetDevice only when it is not
// already (the call costs tens of microseconds even when nothing changes).
hipError_t psgld::use_device(int dev)
{
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur == dev) return hipSuccess;
    return hipSetDevice(dev);
}

namespace {

// Returns one device block of the context to where it came from: the
// caller's dev_free hook, or hipFree.
void release_block(const psgld_ctx *c, void *p, size_t bytes)
{
    if (c->opt.dev_free) c->opt.dev_free(p, bytes, c->opt.alloc_user);
    else (void)hipFree(p);
}

// Every device allocation of a context: through the caller's hooks when
// the options give them, else hipMalloc.  Sizes are recorded per block.
template <typename T>
psgld_status dev_alloc(psgld_ctx *c, T **p, size_t count)
{
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (c->opt.dev_alloc) {
        q = c->opt.dev_alloc(bytes, c->opt.alloc_user);
        if (!q) return c->fail(PSGLD_E_NOMEM, "allocator hook returned NULL for " + std::to_string(bytes) + " bytes");
        if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {
            c->opt.dev_free(q, bytes, c->opt.alloc_user);
            return c->fail(PSGLD_E_ARG, "allocator hook returned memory not aligned to 256 bytes");
        }
    } else if (hipMalloc(&q, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return c->fail(PSGLD_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    c->allocs.emplace(q, bytes);
    c->bytes += static_cast<int64_t>(bytes);
    *p = static_cast<T *>(q);
    return PSGLD_OK;
}

void dev_free(psgld_ctx *c, void *p)
{
    if (!p) return;
    auto it = c->allocs.find(p);
    if (it == c->allocs.end()) return;
    const size_t bytes = it->second;
    c->allocs.erase(it);
    c->bytes -= static_cast<int64_t>(bytes);
    release_block(c, p, bytes);
}

// Destroys every captured graph (after the work already enqueued has run).
void drop_graphs(psgld_ctx *c)
{
    if (c->graphs.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
}

psgld_status ensure_device(psgld_ctx *c)
{
    if (c->device_ready) return PSGLD_OK;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= c->opt.device) {
        (void)hipGetLastError();
        return c->fail(PSGLD_E_DEVICE, "no HIP device " + std::to_string(c->opt.device));
    }
    HIPTRY(c, use_device(c->opt.device));
    if (!is_gfx950(c->opt.device)) return c->fail(PSGLD_E_DEVICE, "device is not gfx950 (MI355X)");
    if (c->opt.stream) {
        c->stream = static_cast<hipStream_t>(c->opt.stream);
    } else {
        HIPTRY(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    psgld_status s = dev_alloc(c, &c->nonfinite, 1);
    if (!s) s = dev_alloc(c, &c->clock, 1);
    if (!s) s = dev_alloc(c, &c->barrier, 1);
    if (s) {
        // nothing else exists yet: return what was allocated and the stream
        for (auto &blk : c->allocs) release_block(c, blk.first, blk.second);
        c->allocs.clear();
        c->bytes = 0;
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        c->stream = nullptr;
        c->own_stream = false;
        return s;
    }
    const int32_t big = INT_MAX;
    HIPTRY(c, hipMemcpy(c->nonfinite, &big, sizeof(big), hipMemcpyHostToDevice));
    c->device_ready = true;
    return PSGLD_OK;
}

template <typename T>
psgld_status upload(psgld_ctx *c, T **dst, const std::vector<T> &src)
{
    psgld_status s = dev_alloc(c, dst, src.size());
    if (s) return s;
    if (!src.empty())
        HIPTRY(c, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return PSGLD_OK;
}

int32_t part_of(const psgld_ctx *c, int32_t i, int32_t j)
{
    return (c->col_piece[j] - c->row_piece[i] + c->B) % c->B;
}

// s_p = N / n_p in FP64, rounded once (0 for a part without entries).
float part_scale(const psgld_ctx *c, int32_t p)
{
    return c->n_p[p] > 0 ? static_cast<float>(static_cast<double>(c->N) / static_cast<double>(c->n_p[p])) : 0.f;
}

// Part of iteration t: t mod B, or drawn with probability n_p / N (random
// order; the rule is documented with PSGLD_PART_RANDOM).
int32_t part_at(const psgld_ctx *c, int64_t t)
{
    if (c->opt.part_order != PSGLD_PART_RANDOM || c->N <= 0) return static_cast<int32_t>(t % c->B);
    const Block4 r = philox4x32_10(0u, 0u, static_cast<uint32_t>(t), 4u, static_cast<uint32_t>(c->opt.seed),
                                   static_cast<uint32_t>(c->opt.seed >> 32));
    const uint64_t lhs = (2ull * (r.r[0] >> 9) + 1ull) * static_cast<uint64_t>(c->N);
    uint64_t cum = 0;
    for (int32_t p = 0; p < c->B; ++p) {
        cum += static_cast<uint64_t>(c->n_p[p]);
        if (lhs < (cum << 24)) return p;
    }
    return c->B - 1;
}

// Builds every part's work schedule for c->sched and uploads it, replacing
// any previous one.
psgld_status upload_schedule(psgld_ctx *c)
{
    const int64_t I = c->I, J = c->J;
    const int32_t B = c->B;
    std::vector<WgTask> tasks;
    std::vector<GroupRec> recs;
    int32_t max_splits = 0;
    c->task_off.assign(B, 0);
    c->n_tasks.assign(B, 0);
    for (int32_t p = 0; p < B; ++p) {
        PartSchedule ps;
        build_part_schedule(c->pre_r.data() + static_cast<size_t>(p) * I, c->pre_c.data() + static_cast<size_t>(p) * J,
                            I, J, c->row_piece, c->col_piece, B, p, c->lpg, c->sched,
                            c->skip.empty() ? nullptr : c->skip.data() + static_cast<size_t>(p) * B, ps);
        c->task_off[p] = static_cast<int64_t>(tasks.size());
        c->n_tasks[p] = static_cast<int64_t>(ps.tasks.size());
        tasks.insert(tasks.end(), ps.tasks.begin(), ps.tasks.end());
        recs.insert(recs.end(), ps.recs.begin(), ps.recs.end());
        max_splits = std::max(max_splits, ps.n_splits);
    }
    HIPTRY(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    dev_free(c, c->tasks);
    dev_free(c, c->recs);
    dev_free(c, c->split_partial);
    dev_free(c, c->split_count);
    c->tasks = nullptr;
    c->recs = nullptr;
    c->split_partial = nullptr;
    c->split_count = nullptr;
    psgld_status s;
    if ((s = upload(c, &c->tasks, tasks))) return s;
    if ((s = upload(c, &c->recs, recs))) return s;
    std::vector<int32_t> toff(B), ntk(B);
    c->max_tasks = 0;
    for (int32_t p = 0; p < B; ++p) {
        toff[p] = static_cast<int32_t>(c->task_off[p]);
        ntk[p] = static_cast<int32_t>(c->n_tasks[p]);
        c->max_tasks = std::max(c->max_tasks, ntk[p]);
    }
    dev_free(c, c->task_off_dev);
    dev_free(c, c->n_tasks_dev);
    c->task_off_dev = c->n_tasks_dev = nullptr;
    if ((s = upload(c, &c->task_off_dev, toff))) return s;
    if ((s = upload(c, &c->n_tasks_dev, ntk))) return s;
    c->job_valid = false;
    c->max_splits = max_splits;
    if ((s = dev_alloc(c, &c->split_partial, static_cast<size_t>(max_splits) * c->Kp))) return s;
    if ((s = dev_alloc(c, &c->split_count, static_cast<size_t>(max_splits)))) return s;
    HIPTRY(c, hipMemset(c->split_count, 0, std::max<int32_t>(max_splits, 1) * sizeof(int32_t)));
    return PSGLD_OK;
}

// Shape signature of a context for the tuning cache: sizes, rank, blocks,
// likelihood branch and the longest row and column of any part.
std::string tune_key(const psgld_ctx *c)
{
    int32_t max_r = 0, max_c = 0;
    for (size_t k = 0; k + 1 < c->pre_r.size(); ++k) max_r = std::max(max_r, c->pre_r[k + 1] - c->pre_r[k]);
    for (size_t k = 0; k + 1 < c->pre_c.size(); ++k) max_c = std::max(max_c, c->pre_c[k + 1] - c->pre_c[k]);
    char buf[256];
    std::snprintf(buf, sizeof(buf), "gfx950:I%lld:J%lld:K%d:B%d:N%lld:lik%d:r%d:c%d", static_cast<long long>(c->I),
                  static_cast<long long>(c->J), c->K, c->B, static_cast<long long>(c->N), c->lik_kind, max_r, max_c);
    return buf;
}

// A tuned schedule: entries per lane group and quads per lane (which sets
// the lanes per group).
struct TuneChoice {
    int entries_per_group = 0;
    int qpl = 0;
};

std::mutex g_tune_mutex;
std::map<std::string, TuneChoice> g_tune_memo;

// The choice remembered for this signature in this process, else in the
// file named by PSGLD_TUNE_CACHE (lines "<signature> <entries per group>
// <quads per lane>"), else none (entries_per_group 0).
TuneChoice cached_choice(const psgld_ctx *c)
{
    const std::string key = tune_key(c);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune_memo.find(key);
    if (it != g_tune_memo.end()) return it->second;
    TuneChoice found;
    if (const char *path = std::getenv("PSGLD_TUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "r")) {
            char k[256];
            int v = 0, q = 0;
            while (std::fscanf(f, "%255s %d %d", k, &v, &q) == 3)
                if (key == k && v > 0 && sparse_variant_exists(sparse_lanes_for(c->K, q), q)) found = TuneChoice{v, q};
            std::fclose(f);
            if (found.entries_per_group > 0) g_tune_memo[key] = found;
        }
    }
    return found;
}

void remember_choice(const psgld_ctx *c, TuneChoice value)
{
    const std::string key = tune_key(c);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_memo[key] = value;
    if (const char *path = std::getenv("PSGLD_TUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%s %d %d\n", key.c_str(), value.entries_per_group, value.qpl);
            std::fclose(f);
        }
    }
}

// Sets the quads per lane (and so the lanes per group) of the sparse kernels.
void set_variant(psgld_ctx *c, int qpl)
{
    c->qpl = qpl;
    c->lpg = sparse_lanes_for(c->K, qpl);
}

// Builds and uploads the part-major layout from training coordinates.
psgld_status build_layout(psgld_ctx *c, int64_t nnz, const int32_t *row, const int32_t *col,
                          const float *val)
{
    if (nnz < 0 || nnz > kMaxEntries)
        return c->fail(PSGLD_E_ARG, "at most 2^31 - 64 training entries are held as coordinates");
    const int64_t I = c->I, J = c->J;
    const int32_t B = c->B;
    // bucket by (part, row) and by (part, column): counting sort
    std::vector<int32_t> part(nnz);
    for (int64_t e = 0; e < nnz; ++e) part[e] = part_of(c, row[e], col[e]);
    std::vector<int32_t> pre_r(static_cast<size_t>(B) * I + 1, 0), pre_c(static_cast<size_t>(B) * J + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) {
        pre_r[static_cast<size_t>(part[e]) * I + row[e] + 1]++;
        pre_c[static_cast<size_t>(part[e]) * J + col[e] + 1]++;
    }
    for (size_t k = 1; k < pre_r.size(); ++k) pre_r[k] += pre_r[k - 1];
    for (size_t k = 1; k < pre_c.size(); ++k) pre_c[k] += pre_c[k - 1];
    std::vector<Entry> er(nnz), ec(nnz);
    std::vector<int32_t> rows_of(nnz);
    {
        std::vector<int32_t> fr(pre_r.begin(), pre_r.end() - 1), fc(pre_c.begin(), pre_c.end() - 1);
        for (int64_t e = 0; e < nnz; ++e) {
            const int32_t kr = fr[static_cast<size_t>(part[e]) * I + row[e]]++;
            er[kr] = Entry{col[e], val[e]};
            rows_of[kr] = row[e];
            const int32_t kc = fc[static_cast<size_t>(part[e]) * J + col[e]]++;
            ec[kc] = Entry{row[e], val[e]};
        }
    }
    auto by_idx = [](const Entry &a, const Entry &b) { return a.off < b.off; };
    for (size_t k = 0; k + 1 < pre_r.size(); ++k) {
        if (pre_r[k + 1] - pre_r[k] > 1) {
            std::sort(er.begin() + pre_r[k], er.begin() + pre_r[k + 1], by_idx);
            for (int32_t m = pre_r[k] + 1; m < pre_r[k + 1]; ++m)
                if (er[m].off == er[m - 1].off) {
                    const int64_t i = static_cast<int64_t>(k % I);
                    return c->fail(PSGLD_E_ARG, "duplicate training entry (" + std::to_string(i) +
                                                    ", " + std::to_string(er[m].off) + ")");
                }
        }
    }
    for (size_t k = 0; k + 1 < pre_c.size(); ++k)
        if (pre_c[k + 1] - pre_c[k] > 1) std::sort(ec.begin() + pre_c[k], ec.begin() + pre_c[k + 1], by_idx);
    // partner indices -> offsets into the factor arrays; pad the arrays
    for (auto &x : er) x.off *= c->Kp;
    for (auto &x : ec) x.off *= c->Kp;
    er.resize(static_cast<size_t>(nnz) + kEntryPad, Entry{0, 0.f});
    ec.resize(static_cast<size_t>(nnz) + kEntryPad, Entry{0, 0.f});

    c->N = nnz;
    c->nnz_sparse = nnz;
    c->n_p.assign(B, 0);
    for (int32_t p = 0; p < B; ++p) c->n_p[p] = pre_r[static_cast<size_t>(p + 1) * I] - pre_r[static_cast<size_t>(p) * I];

    psgld_status s;
    if ((s = upload(c, &c->rowptr, pre_r))) return s;
    if ((s = upload(c, &c->colptr, pre_c))) return s;
    if ((s = upload(c, &c->ent_r, er))) return s;
    if ((s = upload(c, &c->ent_c, ec))) return s;
    if ((s = upload(c, &c->row_of_entry, rows_of))) return s;

    const size_t nw = static_cast<size_t>(I) * c->Kp, nh = static_cast<size_t>(J) * c->Kp;
    for (int b = 0; b < 2; ++b) {
        if ((s = dev_alloc(c, &c->W[b], nw + kFactorPad))) return s;
        if ((s = dev_alloc(c, &c->H[b], nh + kFactorPad))) return s;
        HIPTRY(c, hipMemset(c->W[b], 0, (nw + kFactorPad) * sizeof(float)));
        HIPTRY(c, hipMemset(c->H[b], 0, (nh + kFactorPad) * sizeof(float)));
    }
    for (int side = 0; side < 2; ++side) {
        const size_t n = side == 0 ? nw : nh;
        if ((s = dev_alloc(c, &c->sum[side], n))) return s;
        if ((s = dev_alloc(c, &c->sum2[side], n))) return s;
        HIPTRY(c, hipMemset(c->sum[side], 0, n * sizeof(double)));
        HIPTRY(c, hipMemset(c->sum2[side], 0, n * sizeof(double)));
    }
    c->ll_blocks = 1024;
    if ((s = dev_alloc(c, &c->ll_partials, c->ll_blocks))) return s;
    if ((s = dev_alloc(c, &c->ll_out, 1))) return s;
    c->part_visits.assign(B, 0);
    c->pre_r.swap(pre_r);
    c->pre_c.swap(pre_c);
    const TuneChoice tc = cached_choice(c);
    if (tc.entries_per_group > 0) {
        c->sched.entries_per_group = tc.entries_per_group;
        set_variant(c, tc.qpl);
    }
    if ((s = upload_schedule(c))) return s;
    c->loaded = true;
    return PSGLD_OK;
}

int32_t dense_slot_rows(const psgld_ctx *c) { return (c->dense_max_m + 31) / 32 * 32; }

// Dense products on BF16 operands (both BF16 precisions).
bool bf16_operands(const psgld_ctx *c) { return c->opt.precision != PSGLD_FP32; }

// FP32 -> BF16, rounded to nearest even (values are finite: checked on load).
uint16_t bf16_round(float v)
{
    uint32_t u;
    std::memcpy(&u, &v, sizeof u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

// Rows of a dense block's MFMA tiles are padded to this: the k-depth of one
// MFMA step over rows (4 for FP32 operands, 32 for BF16), rounded to 16.
int dense_row_align(const psgld_ctx *c) { return bf16_operands(c) ? 32 : 16; }

// Sub-tiles per work-group for a block of m rows: the four waves of a
// work-group share a sub-tile's 16-row tiles, so a block of up to 64 (padded)
// rows gives each wave one tile per sub-tile and takes four sub-tiles, a
// taller one two tiles per wave and takes two -- the work-groups of the
// tallest block, which set when the launch ends (all of them run at once),
// then have about the work of the others.
int dense_sub_tiles(int m, int row_align)
{
    const int MT = (m + row_align - 1) / row_align * row_align;
    const int tiles_per_wave = (MT + 63) / 64;
    return std::max(1, kDenseSubTiles / tiles_per_wave);
}

psgld_status check_values(psgld_ctx *c, int64_t n, const float *val)
{
    for (int64_t e = 0; e < n; ++e) {
        const float v = val[e];
        if (!std::isfinite(v)) return c->fail(PSGLD_E_ARG, "non-finite value at entry " + std::to_string(e));
        if (c->lik.beta <= 1.0 && v < 0.f)
            return c->fail(PSGLD_E_ARG, "negative value at entry " + std::to_string(e) + " with beta <= 1");
        if (c->lik.beta <= 0.0 && v <= 0.f)
            return c->fail(PSGLD_E_ARG, "non-positive value at entry " + std::to_string(e) + " with beta <= 0");
    }
    return PSGLD_OK;
}

psgld_status check_coords(psgld_ctx *c, int64_t n, const int32_t *row, const int32_t *col)
{
    for (int64_t e = 0; e < n; ++e) {
        if (row[e] < 0 || row[e] >= c->I || col[e] < 0 || col[e] >= c->J)
            return c->fail(PSGLD_E_ARG, "coordinate out of range at entry " + std::to_string(e));
    }
    return PSGLD_OK;
}

psgld_status sync_and_check(psgld_ctx *c)
{
    if (!c->device_ready) return PSGLD_OK;
    HIPTRY(c, use_device(c->opt.device));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    int32_t flag = INT_MAX;
    HIPTRY(c, hipMemcpy(&flag, c->nonfinite, sizeof(flag), hipMemcpyDeviceToHost));
    if (flag != INT_MAX)
        return c->fail(PSGLD_E_NUMERIC, "non-finite value in W or H at iteration " + std::to_string(flag));
    return PSGLD_OK;
}

// Device FP32 factor (rows x Kp) -> host rows x K, optionally transposed to K x rows.
template <typename TOut, typename TDev>
psgld_status fetch_factor(psgld_ctx *c, const TDev *dev, int64_t rows, bool transpose, TOut *out,
                          double scale)
{
    std::vector<TDev> tmp(static_cast<size_t>(rows) * c->Kp);
    HIPTRY(c, hipMemcpy(tmp.data(), dev, tmp.size() * sizeof(TDev), hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < rows; ++r)
        for (int32_t k = 0; k < c->K; ++k) {
            const TOut v = static_cast<TOut>(static_cast<double>(tmp[static_cast<size_t>(r) * c->Kp + k]) * scale);
            if (transpose) out[static_cast<size_t>(k) * rows + r] = v;
            else out[static_cast<size_t>(r) * c->K + k] = v;
        }
    return PSGLD_OK;
}

// Makes the device step-size table cover iterations [t_begin, t_end) for
// `sched`.  Refilling waits for the enqueued work; moving or reallocating
// the table drops the captured graphs, which hold its address.
psgld_status ensure_eps_table(psgld_ctx *c, const psgld_eps_schedule *sched, int64_t t_begin, int64_t t_end)
{
    const bool same = c->eps_tab && sched->a == c->eps_sched.a && sched->t0 == c->eps_sched.t0 &&
                      sched->gamma == c->eps_sched.gamma;
    if (same && t_begin >= c->eps_base && t_end <= c->eps_base + c->eps_cap) return PSGLD_OK;
    HIPTRY(c, hipStreamSynchronize(c->stream));
    int64_t base = c->eps_base, cap = c->eps_cap;
    if (!c->eps_tab || t_begin < base || t_end > base + cap) {
        base = t_begin;
        cap = 4096;
        while (cap < 2 * (t_end - t_begin)) cap *= 2;
        drop_graphs(c);
        dev_free(c, c->eps_tab);
        dev_free(c, c->part_tab);
        c->eps_tab = nullptr;
        c->part_tab = nullptr;
        psgld_status s = dev_alloc(c, &c->eps_tab, static_cast<size_t>(cap));
        if (!s && c->opt.part_order == PSGLD_PART_RANDOM) s = dev_alloc(c, &c->part_tab, static_cast<size_t>(cap));
        if (s) return s;
    }
    std::vector<float2> tab(static_cast<size_t>(cap));
    for (int64_t k = 0; k < cap; ++k) {
        const double eps = sched->a * std::pow(sched->t0 + static_cast<double>(base + k), -sched->gamma);
        tab[k] = make_float2(static_cast<float>(eps), static_cast<float>(std::sqrt(2.0 * eps)));
    }
    HIPTRY(c, hipMemcpy(c->eps_tab, tab.data(), tab.size() * sizeof(float2), hipMemcpyHostToDevice));
    if (c->part_tab) {
        std::vector<int32_t> parts(static_cast<size_t>(cap));
        for (int64_t k = 0; k < cap; ++k) parts[k] = part_at(c, base + k);
        HIPTRY(c, hipMemcpy(c->part_tab, parts.data(), parts.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    c->eps_base = base;
    c->eps_cap = cap;
    c->eps_sched = *sched;
    return PSGLD_OK;
}

// Enqueues one iteration of part p reading ping-pong buffer `cur`.  The
// iteration index is *clock + k when clock is given (captured graphs), else
// k.  With bookkeeping off (tuning trials) no moments or held-out sums are
// touched.
// Device buffers an iteration reads beside the context's own arrays: the
// step-size table (indexed by the global iteration) and the scratch of items
// cut over several work-groups.  Null: the context's.
struct IterBuffers {
    const float2 *eps_tab;
    float *split_partial;
    int32_t *split_count;
};

hipError_t enqueue_iteration(psgld_ctx *c, int32_t p, int cur, const int32_t *clock, int32_t k, bool bookkeeping,
                             hipStream_t stream, const IterBuffers *buf = nullptr)
{
    const int64_t I = c->I, J = c->J;
    IterClock clk{};
    clk.eps_tab = buf ? buf->eps_tab : c->eps_tab - c->eps_base;   // indexed by the global iteration
    clk.clock = clock;
    clk.k = k;
    clk.burn_in = static_cast<int32_t>(std::min<int64_t>(c->opt.burn_in, INT32_MAX));
    clk.thin = c->opt.thin;
    clk.bookkeeping = bookkeeping ? 1 : 0;
    SparseIterArgs a{};
    a.x_old[0] = c->W[cur];
    a.x_old[1] = c->H[cur];
    a.x_new[0] = c->W[cur ^ 1];
    a.x_new[1] = c->H[cur ^ 1];
    a.ptr[0] = c->rowptr + static_cast<size_t>(p) * I;
    a.ptr[1] = c->colptr + static_cast<size_t>(p) * J;
    a.ent[0] = c->ent_r;
    a.ent[1] = c->ent_c;
    a.tasks = c->tasks + c->task_off[p];
    a.recs = c->recs + static_cast<size_t>(c->task_off[p]) * (sparse_block_threads() / c->lpg);
    a.n_tasks = static_cast<int32_t>(c->n_tasks[p]);
    a.split_partial = buf ? buf->split_partial : c->split_partial;
    a.split_count = buf ? buf->split_count : c->split_count;
    a.K = c->K;
    a.Kp = c->Kp;
    a.nq = c->nq;
    a.scale = part_scale(c, p);
    a.lambda[0] = static_cast<float>(c->prior.lambda_w);
    a.lambda[1] = static_cast<float>(c->prior.lambda_h);
    a.inv_phi = static_cast<float>(1.0 / c->lik.phi);
    a.beta = static_cast<float>(c->lik.beta);
    a.mu_floor = static_cast<float>(c->opt.mu_floor);
    a.seed_lo = static_cast<uint32_t>(c->opt.seed);
    a.seed_hi = static_cast<uint32_t>(c->opt.seed >> 32);
    a.mirror = c->prior.mirror ? 1 : 0;
    a.prior_kind = c->prior.kind;
    a.flags = c->opt.test_flags;
    a.clk = clk;
    a.clk.has_heldout = c->n_ho > 0 ? 1 : 0;
    for (int side = 0; side < 2; ++side) {
        a.sum[side] = c->sum[side];
        a.sum2[side] = c->sum2[side];
    }
    a.ho_ptr = c->ho_ptr ? c->ho_ptr + static_cast<size_t>(p) * I : nullptr;
    a.ho_ent = c->ho_ent;
    a.ho_sum = c->ho_sum;
    a.nonfinite = c->nonfinite;
    hipError_t e = launch_sparse_iter(a, c->lik_kind, c->lpg, c->qpl, stream);
    if (e != hipSuccess) return e;
    if (!c->dblocks_host.empty() && c->dblk_cnt[p] > 0) {
        DenseIterArgs d{};
        d.x_old[0] = a.x_old[0];
        d.x_old[1] = a.x_old[1];
        d.x_new[0] = a.x_new[0];
        d.x_new[1] = a.x_new[1];
        d.blocks = c->dblocks + c->dblk_off[p];
        d.n_blocks = static_cast<int32_t>(c->dblk_cnt[p]);
        d.tiles = c->dtiles + c->dtile_off[p];
        d.n_tiles = static_cast<int32_t>(c->dtile_cnt[p]);
        d.val = c->dval;
        d.val16 = c->dval16;
        d.mask = c->dmask;
        d.w_partial = c->w_partial;
        d.slot_rows = dense_slot_rows(c);
        d.row_align = dense_row_align(c);
        d.K = c->K;
        d.Kp = c->Kp;
        d.KS = c->KS;
        d.scale = a.scale;
        d.lambda[0] = a.lambda[0];
        d.lambda[1] = a.lambda[1];
        d.inv_phi = a.inv_phi;
        d.beta = a.beta;
        d.mu_floor = a.mu_floor;
        d.seed_lo = a.seed_lo;
        d.seed_hi = a.seed_hi;
        d.mirror = a.mirror;
        d.prior_kind = a.prior_kind;
        d.flags = a.flags;
        d.clk = clk;
        d.clk.has_heldout = c->dheld != nullptr ? 1 : 0;
        for (int side = 0; side < 2; ++side) {
            d.sum[side] = a.sum[side];
            d.sum2[side] = a.sum2[side];
        }
        d.heldout = c->dheld;
        d.ho_sum = c->ho_sum;
        d.nonfinite = c->nonfinite;
        e = launch_dense_iter(d, c->lik_kind, bf16_operands(c), c->dense_max_m, stream);
    }
    return e;
}

// Host-side record of iteration t having been enqueued with bookkeeping on:
// kept samples and the visits of each part after burn-in.
void account_iteration(psgld_ctx *c, int64_t t)
{
    if (t < c->opt.burn_in) return;
    if ((t - c->opt.burn_in) % c->opt.thin == 0) c->n_kept++;
    if (c->n_ho > 0) c->part_visits[part_at(c, t)]++;
}

// Iterations per captured graph (0 = do not capture).
int64_t graph_length(const psgld_ctx *c)
{
    if (c->opt.graph_iters < 0 || c->opt.part_order == PSGLD_PART_RANDOM) return 0;
    if (c->opt.graph_iters > 0) return c->opt.graph_iters;
    return static_cast<int64_t>(c->B) * ((32 + c->B - 1) / c->B);
}

// The graph of L iterations starting at part r from buffer cur, captured on
// first use: the iterations read t from the device clock, then the clock
// advances by L.
psgld_status get_graph(psgld_ctx *c, int32_t r, int cur, int64_t L, hipGraphExec_t *out)
{
    const auto key = std::make_tuple(r, cur, L);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return PSGLD_OK;
    }
    // the capture stream is created on first capture: creating a stream costs
    // about a millisecond, which contexts that never capture should not pay
    if (!c->cap_stream) HIPTRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPTRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int64_t k = 0; k < L && e == hipSuccess; ++k)
        e = enqueue_iteration(c, static_cast<int32_t>((r + k) % c->B), static_cast<int>((cur + k) & 1), c->clock,
                              static_cast<int32_t>(k), true, c->cap_stream);
    if (e == hipSuccess) e = launch_advance_clock(c->clock, static_cast<int32_t>(L), c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e_end = hipStreamEndCapture(c->cap_stream, &graph);
    if (e == hipSuccess) e = e_end;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return c->fail(PSGLD_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
    }
    c->graphs[key] = exec;
    *out = exec;
    return PSGLD_OK;
}

// The context as the batched kernel reads it; uploaded when it changed
// (after the work already enqueued has run).
psgld_status sync_job_desc(psgld_ctx *c)
{
    JobDesc d{};
    for (int b = 0; b < 2; ++b) {
        d.W[b] = c->W[b];
        d.H[b] = c->H[b];
    }
    d.rowptr = c->rowptr;
    d.colptr = c->colptr;
    d.ent[0] = c->ent_r;
    d.ent[1] = c->ent_c;
    d.tasks = c->tasks;
    d.recs = c->recs;
    d.task_off = c->task_off_dev;
    d.n_tasks = c->n_tasks_dev;
    d.scale = c->scale_dev;
    d.split_partial = c->split_partial;
    d.split_count = c->split_count;
    d.I = static_cast<int32_t>(c->I);
    d.J = static_cast<int32_t>(c->J);
    d.K = c->K;
    d.Kp = c->Kp;
    d.nq = c->nq;
    d.B = c->B;
    d.lambda[0] = static_cast<float>(c->prior.lambda_w);
    d.lambda[1] = static_cast<float>(c->prior.lambda_h);
    d.inv_phi = static_cast<float>(1.0 / c->lik.phi);
    d.beta = static_cast<float>(c->lik.beta);
    d.mu_floor = static_cast<float>(c->opt.mu_floor);
    d.seed_lo = static_cast<uint32_t>(c->opt.seed);
    d.seed_hi = static_cast<uint32_t>(c->opt.seed >> 32);
    d.mirror = c->prior.mirror ? 1 : 0;
    d.prior_kind = c->prior.kind;
    d.flags = c->opt.test_flags;
    d.eps_tab = c->eps_tab - c->eps_base;
    d.part_tab = c->part_tab ? c->part_tab - c->eps_base : nullptr;
    d.clock = c->clock;
    d.cur_phase = (c->cur ^ static_cast<int>(c->t & 1)) & 1;
    d.burn_in = static_cast<int32_t>(std::min<int64_t>(c->opt.burn_in, INT32_MAX));
    d.thin = c->opt.thin;
    d.has_heldout = c->n_ho > 0 ? 1 : 0;
    for (int side = 0; side < 2; ++side) {
        d.sum[side] = c->sum[side];
        d.sum2[side] = c->sum2[side];
    }
    d.ho_ptr = c->ho_ptr;
    d.ho_ent = c->ho_ent;
    d.ho_sum = c->ho_sum;
    d.nonfinite = c->nonfinite;
    if (c->job_valid && std::memcmp(&d, &c->job_host, sizeof(d)) == 0) return PSGLD_OK;
    HIPTRY(c, hipStreamSynchronize(c->stream));
    if (!c->job_desc) {
        std::vector<float> scl(c->B);
        for (int32_t p = 0; p < c->B; ++p) scl[p] = part_scale(c, p);
        psgld_status s = dev_alloc(c, &c->job_desc, 1);
        if (!s) s = upload(c, &c->scale_dev, scl);
        if (s) return s;
        d.scale = c->scale_dev;
    }
    HIPTRY(c, hipMemcpy(c->job_desc, &d, sizeof(d), hipMemcpyHostToDevice));
    c->job_host = d;
    c->job_valid = true;
    return PSGLD_OK;
}

// n_iter iterations of coordinate-stored contexts of one kernel variant in
// cooperative launches of up to kPersistentIters iterations, then the host
// record of those iterations.  Step-size tables must cover them.
constexpr int64_t kPersistentIters = 256;

psgld_status step_persistent(psgld_ctx *const *ctxs, int n, int64_t n_iter, hipStream_t stream)
{
    psgld_ctx *c0 = ctxs[0];
    for (int j = 0; j < n; ++j) {
        psgld_ctx *c = ctxs[j];
        psgld_status s = sync_job_desc(c);
        if (s) return s;
        if (c->clock_host != c->t) {
            HIPTRY(c, launch_set_clock(c->clock, static_cast<int32_t>(c->t), stream));
            c->clock_host = c->t;
        }
    }
    for (int first = 0; first < n; first += kMaxBatch) {
        const int cnt = std::min(kMaxBatch, n - first);
        BatchArgs b{};
        b.n = cnt;
        std::vector<int32_t *> clocks;
        for (int q = 0; q < cnt; ++q) {
            psgld_ctx *c = ctxs[first + q];
            b.jobs[q] = c->job_desc;
            b.wg_first[q + 1] = b.wg_first[q] + c->max_tasks;
            clocks.push_back(c->clock);
        }
        for (int64_t done = 0; done < n_iter; done += kPersistentIters) {
            const int chunk = static_cast<int>(std::min(kPersistentIters, n_iter - done));
            HIPTRY(c0, launch_sparse_persistent(b, chunk, c0->lik_kind, c0->lpg, c0->qpl, c0->opt.persistent_grid,
                                                c0->barrier, stream));
            const std::vector<int32_t> delta(clocks.size(), chunk);
            HIPTRY(c0, launch_advance_clocks(clocks.data(), delta.data(), cnt, stream));
        }
    }
    for (int j = 0; j < n; ++j) {
        psgld_ctx *c = ctxs[j];
        for (int64_t k = 0; k < n_iter; ++k) account_iteration(c, c->t + k);
        c->cur ^= static_cast<int>(n_iter & 1);
        c->t += n_iter;
        c->clock_host = c->t;
    }
    return PSGLD_OK;
}

psgld_status check_schedule(psgld_ctx *c, const psgld_eps_schedule *sched)
{
    if (!sched) return c->fail(PSGLD_E_ARG, "schedule is required");
    if (!(sched->a > 0.0) || !std::isfinite(sched->a)) return c->fail(PSGLD_E_ARG, "eps: a must be > 0");
    if (!(sched->gamma == 0.0 || (sched->gamma > 0.5 && sched->gamma <= 1.0)))
        return c->fail(PSGLD_E_ARG, "eps: gamma must be in (0.5, 1] (Eq. (4)) or 0");
    if (sched->gamma > 0.0 && !(sched->t0 > 0.0)) return c->fail(PSGLD_E_ARG, "eps: t0 must be > 0");
    return PSGLD_OK;
}

}  // namespace

extern "C" {

void psgld_default_options(psgld_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->seed = 0;
    opt->burn_in = 0;
    opt->thin = 1;
    opt->precision = PSGLD_FP32;
    opt->dense_threshold = 0.3;
    opt->mu_floor = 1e-6;
    opt->row_piece = nullptr;
    opt->col_piece = nullptr;
    opt->stream = nullptr;
    opt->test_flags = 0;
    opt->device = 0;
    opt->graph_iters = -1;
    opt->persistent = 0;
    opt->part_order = PSGLD_PART_CYCLIC;
    opt->dense_min_cols = 256;
    opt->persistent_grid = 0;
    opt->dev_alloc = nullptr;
    opt->dev_free = nullptr;
    opt->alloc_user = nullptr;
}

psgld_status psgld_create(int64_t I, int64_t J, int32_t K, int32_t B, const psgld_likelihood *lik,
                          const psgld_prior *prior, const psgld_options *opt, psgld_ctx **out)
{
    auto bad = [](const std::string &m) {
        g_create_error = m;
        return PSGLD_E_ARG;
    };
    if (!out) return bad("out is NULL");
    *out = nullptr;
    if (!lik || !prior) return bad("likelihood and prior are required");
    if (I < 1 || J < 1 || I > INT32_MAX || J > INT32_MAX) return bad("I and J must be in [1, 2^31)");
    if (K < 1 || K > 256) return bad("K must be in [1, 256]");
    if ((I + 1) * padded_rank(K) >= INT32_MAX || (J + 1) * padded_rank(K) >= INT32_MAX)
        return bad("I * K and J * K must stay below 2^31");
    if (B < 1 || B > I || B > J) return bad("B must be in [1, min(I, J)]");
    if (!(lik->phi > 0.0) || !std::isfinite(lik->phi) || !std::isfinite(lik->beta)) return bad("phi must be > 0, beta finite");
    if (lik->beta > 1.0 && lik->beta < 2.0) return bad("no Tweedie model exists for 1 < beta < 2");
    if (prior->kind != PSGLD_PRIOR_EXPONENTIAL && prior->kind != PSGLD_PRIOR_GAUSSIAN) return bad("unknown prior kind");
    if (!(prior->lambda_w > 0.0) || !(prior->lambda_h > 0.0)) return bad("prior rates must be > 0");
    psgld_options o;
    psgld_default_options(&o);
    if (opt) o = *opt;
    if (o.thin < 1) return bad("thin must be >= 1");
    if (o.burn_in < 0) return bad("burn_in must be >= 0");
    if (!(o.mu_floor > 0.0)) return bad("mu_floor must be > 0");
    if (o.precision != PSGLD_FP32 && o.precision != PSGLD_BF16_DENSE && o.precision != PSGLD_BF16_DENSE_VALUES)
        return bad("unknown precision");
    if (o.device < 0) return bad("device must be >= 0");
    if (o.part_order != PSGLD_PART_CYCLIC && o.part_order != PSGLD_PART_RANDOM) return bad("unknown part order");
    if (o.dense_min_cols < 1) return bad("dense_min_cols must be >= 1");
    if (o.persistent_grid < 0) return bad("persistent_grid must be >= 0");
    if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr)) return bad("dev_alloc and dev_free go together");

    psgld_ctx *c = new (std::nothrow) psgld_ctx();
    if (!c) {
        g_create_error = "out of host memory";
        return PSGLD_E_NOMEM;
    }
    c->I = I;
    c->J = J;
    c->K = K;
    c->B = B;
    c->Kp = padded_rank(K);
    c->nq = (K + 3) / 4;
    c->lpg = sparse_threads_per_group(K);
    c->qpl = sparse_quads_per_lane(K);
    c->lik = *lik;
    c->prior = *prior;
    c->opt = o;
    c->lik_kind = lik_kind_of(lik->beta);
    // partitions P_B([I]), P_B([J]): given, or contiguous with the first (n mod B) pieces longer
    for (int side = 0; side < 2; ++side) {
        const int64_t n = side == 0 ? I : J;
        const int32_t *given = side == 0 ? o.row_piece : o.col_piece;
        std::vector<int32_t> &pc = side == 0 ? c->row_piece : c->col_piece;
        pc.resize(n);
        if (given) {
            std::vector<int64_t> cnt(B, 0);
            for (int64_t m = 0; m < n; ++m) {
                if (given[m] < 0 || given[m] >= B) {
                    delete c;
                    return bad("piece index out of range");
                }
                pc[m] = given[m];
                cnt[given[m]]++;
            }
            for (int32_t b = 0; b < B; ++b)
                if (cnt[b] == 0) {
                    delete c;
                    return bad("every piece of a partition must be non-empty");
                }
        } else {
            const int64_t base = n / B, extra = n % B;
            int64_t pos = 0;
            for (int32_t b = 0; b < B; ++b)
                for (int64_t m = 0; m < base + (b < extra ? 1 : 0); ++m) pc[pos++] = b;
        }
    }
    c->opt.row_piece = nullptr;
    c->opt.col_piece = nullptr;
    *out = c;
    return PSGLD_OK;
}

psgld_status psgld_load_coo(psgld_ctx *c, int64_t nnz, const int32_t *row, const int32_t *col,
                            const float *val)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (c->loaded) return c->fail(PSGLD_E_STATE, "data already loaded");
    if (nnz < 0 || nnz > kMaxEntries) return c->fail(PSGLD_E_ARG, "nnz must be in [0, 2^31 - 64]");
    if (nnz > 0 && (!row || !col || !val)) return c->fail(PSGLD_E_ARG, "row, col and val are required");
    psgld_status s;
    if ((s = check_coords(c, nnz, row, col))) return s;
    if ((s = check_values(c, nnz, val))) return s;
    if ((s = ensure_device(c))) return s;
    return build_layout(c, nnz, row, col, val);
}

psgld_status psgld_load_dense(psgld_ctx *c, const float *V, const uint8_t *mask)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (c->loaded) return c->fail(PSGLD_E_STATE, "data already loaded");
    if (!V) return c->fail(PSGLD_E_ARG, "V is required");
    const int64_t I = c->I, J = c->J;
    const int32_t B = c->B;
    for (int64_t i = 0; i < I; ++i)
        for (int64_t j = 0; j < J; ++j) {
            const size_t m = static_cast<size_t>(i) * J + j;
            if (mask && !mask[m]) continue;
            psgld_status s = check_values(c, 1, V + m);
            if (s) return c->fail(s, c->err + " (cell " + std::to_string(i) + ", " + std::to_string(j) + ")");
        }
    // Dense blocks need contiguous pieces, at most kDenseMaxRows rows, at
    // least options.dense_min_cols columns, rank at most kDenseMaxK, and a
    // training density above the threshold.
    const bool contiguous = std::is_sorted(c->row_piece.begin(), c->row_piece.end()) &&
                            std::is_sorted(c->col_piece.begin(), c->col_piece.end());
    std::vector<int64_t> r0(B + 1, 0), c0(B + 1, 0);
    for (int64_t i = 0; i < I; ++i) r0[c->row_piece[i] + 1]++;
    for (int64_t j = 0; j < J; ++j) c0[c->col_piece[j] + 1]++;
    for (int32_t b = 0; b < B; ++b) {
        r0[b + 1] += r0[b];
        c0[b + 1] += c0[b];
    }
    std::vector<uint8_t> dense(static_cast<size_t>(B) * B, 0);
    std::vector<int64_t> train(static_cast<size_t>(B) * B, 0);
    if (contiguous && c->K <= kDenseMaxK) {
        for (int32_t b = 0; b < B; ++b)
            for (int32_t cc = 0; cc < B; ++cc) {
                const int64_t m = r0[b + 1] - r0[b], nn = c0[cc + 1] - c0[cc];
                int64_t cnt = 0;
                for (int64_t i = r0[b]; i < r0[b + 1]; ++i)
                    for (int64_t j = c0[cc]; j < c0[cc + 1]; ++j) cnt += mask ? (mask[i * J + j] != 0) : 1;
                train[static_cast<size_t>(b) * B + cc] = cnt;
                dense[static_cast<size_t>(b) * B + cc] =
                    m <= kDenseMaxRows && nn >= c->opt.dense_min_cols &&
                    cnt > c->opt.dense_threshold * static_cast<double>(m * nn);
            }
    }
    // coordinates of the sparse blocks
    std::vector<int32_t> row, col;
    std::vector<float> val;
    for (int64_t i = 0; i < I; ++i)
        for (int64_t j = 0; j < J; ++j) {
            const size_t m = static_cast<size_t>(i) * J + j;
            if (mask && !mask[m]) continue;
            if (dense[static_cast<size_t>(c->row_piece[i]) * B + c->col_piece[j]]) continue;
            row.push_back(static_cast<int32_t>(i));
            col.push_back(static_cast<int32_t>(j));
            val.push_back(V[m]);
        }
    c->skip.assign(static_cast<size_t>(B) * B, 0);
    for (int32_t p = 0; p < B; ++p)
        for (int32_t b = 0; b < B; ++b) c->skip[static_cast<size_t>(p) * B + b] = dense[static_cast<size_t>(b) * B + (b + p) % B];
    psgld_status s;
    if ((s = ensure_device(c))) return s;
    if ((s = build_layout(c, static_cast<int64_t>(row.size()), row.data(), col.data(), val.data()))) return s;

    // dense storage, part-major: values, cell codes, block table, tiles
    const int row_align = dense_row_align(c);
    std::vector<float> dv;
    std::vector<uint32_t> &dcodes = c->dcodes_host;
    dcodes.clear();
    std::vector<DenseTile> tiles;
    c->dblock_of.assign(static_cast<size_t>(B) * B, -1);
    c->dblocks_host.clear();
    c->dblock_first_tile.clear();
    c->dmask_host.clear();
    c->dblk_off.assign(B, 0);
    c->dblk_cnt.assign(B, 0);
    c->dtile_off.assign(B, 0);
    c->dtile_cnt.assign(B, 0);
    int64_t max_partial_slots = 0;
    c->dense_max_m = 0;
    for (int32_t p = 0; p < B; ++p) {
        c->dblk_off[p] = static_cast<int64_t>(c->dblocks_host.size());
        c->dtile_off[p] = static_cast<int64_t>(tiles.size());
        int32_t partial = 0;
        for (int32_t b = 0; b < B; ++b) {
            const int32_t cc = (b + p) % B;
            if (!dense[static_cast<size_t>(b) * B + cc]) continue;
            DenseBlock blk;
            blk.row0 = static_cast<int32_t>(r0[b]);
            blk.m = static_cast<int32_t>(r0[b + 1] - r0[b]);
            blk.col0 = static_cast<int32_t>(c0[cc]);
            blk.n = static_cast<int32_t>(c0[cc + 1] - c0[cc]);
            blk.ld = (blk.n + kDenseRowAlign - 1) / kDenseRowAlign * kDenseRowAlign;
            blk.n_sub = dense_sub_tiles(blk.m, row_align);
            blk.v_off = static_cast<int64_t>(dv.size());

            blk.first_partial = partial;
            const int32_t wg_cols = kDenseTileCols * blk.n_sub;
            blk.n_tiles = (blk.n + wg_cols - 1) / wg_cols;
            const int32_t idx_in_part = static_cast<int32_t>(c->dblocks_host.size() - c->dblk_off[p]);
            for (int32_t tt = 0; tt < blk.n_tiles; ++tt)
                tiles.push_back(DenseTile{idx_in_part, tt * wg_cols, partial + tt, {}});
            partial += blk.n_tiles;
            for (int64_t i = 0; i < blk.m; ++i) {
                for (int64_t j = 0; j < blk.n; ++j) {
                    const size_t m = static_cast<size_t>(blk.row0 + i) * J + blk.col0 + j;
                    const uint8_t t = mask ? (mask[m] != 0) : 1;
                    dv.push_back(t ? V[m] : 0.f);
                    c->dmask_host.push_back(t);
                    if (t) {
                        const size_t cell = dv.size() - 1;
                        if (dcodes.size() <= cell / 16) dcodes.resize(cell / 16 + 1, 0u);
                        dcodes[cell / 16] |= uint32_t{kMaskTrain} << (2 * (cell % 16));
                    }
                }
                dv.resize(dv.size() + (blk.ld - blk.n), 0.f);
                c->dmask_host.resize(c->dmask_host.size() + (blk.ld - blk.n), 0);
            }
            c->dense_max_m = std::max(c->dense_max_m, blk.m);
            c->dblock_first_tile.push_back(static_cast<int64_t>(tiles.size()) - blk.n_tiles);
            c->dblock_of[static_cast<size_t>(b) * B + cc] = static_cast<int32_t>(c->dblocks_host.size());
            c->dblocks_host.push_back(blk);
            c->N += train[static_cast<size_t>(b) * B + cc];
            c->n_p[p] += train[static_cast<size_t>(b) * B + cc];
        }
        c->dblk_cnt[p] = static_cast<int64_t>(c->dblocks_host.size()) - c->dblk_off[p];
        c->dtile_cnt[p] = static_cast<int64_t>(tiles.size()) - c->dtile_off[p];
        max_partial_slots = std::max<int64_t>(max_partial_slots, partial);
    }
    if (!c->dblocks_host.empty()) {
        const int align = bf16_operands(c) ? 32 : 16;
        c->KS = (c->K + align - 1) / align * align;
        HIPTRY(c, dense_prepare(c->dense_max_m, c->KS));
        if ((s = upload(c, &c->dblocks, c->dblocks_host))) return s;
        if ((s = upload(c, &c->dtiles, tiles))) return s;
        c->dtiles_host = tiles;
        if (c->opt.precision == PSGLD_BF16_DENSE_VALUES) {
            std::vector<uint16_t> dv16(dv.size());
            for (size_t k = 0; k < dv.size(); ++k) dv16[k] = bf16_round(dv[k]);
            if ((s = upload(c, &c->dval16, dv16))) return s;
        } else if ((s = upload(c, &c->dval, dv))) {
            return s;
        }
        dcodes.resize((dv.size() + 15) / 16, 0u);
        if ((s = upload(c, &c->dmask, dcodes))) return s;
        // one slot per tile, each as tall as the tallest padded block
        if ((s = dev_alloc(c, &c->w_partial, static_cast<size_t>(max_partial_slots) * dense_slot_rows(c) * c->Kp)))
            return s;
        // the log-likelihood reduction also covers the dense blocks
        dev_free(c, c->ll_partials);
        c->ll_partials = nullptr;
        if ((s = dev_alloc(c, &c->ll_partials, c->ll_blocks + c->dblocks_host.size() * kDenseLLPerBlock))) return s;
    }
    return PSGLD_OK;
}

psgld_status psgld_load_heldout(psgld_ctx *c, int64_t n, const int32_t *row, const int32_t *col,
                                const float *val)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->loaded) return c->fail(PSGLD_E_STATE, "load training data first");
    if (c->heldout_loaded) return c->fail(PSGLD_E_STATE, "held-out cells already loaded");
    if (c->t > 0) return c->fail(PSGLD_E_STATE, "held-out cells must be loaded before the first step");
    drop_graphs(c);
    if (n < 0 || n >= INT32_MAX) return c->fail(PSGLD_E_ARG, "n must be in [0, 2^31)");
    if (n > 0 && (!row || !col)) return c->fail(PSGLD_E_ARG, "row and col are required");
    psgld_status s;
    if ((s = check_coords(c, n, row, col))) return s;
    if (val)
        for (int64_t e = 0; e < n; ++e)
            if (!std::isfinite(val[e])) return c->fail(PSGLD_E_ARG, "non-finite held-out value");
    const int64_t I = c->I;
    const int32_t B = c->B;
    std::vector<int32_t> pre(static_cast<size_t>(B) * I + 1, 0);
    c->ho_part.resize(n);
    // cells inside dense blocks are summed by the dense kernel's work-group
    // that covers them
    std::vector<uint8_t> in_dense(n, 0);
    std::vector<std::vector<DenseHeld>> dh(c->dtiles_host.size());
    std::vector<uint8_t> held_mark;   // cells of dense blocks seen in this list
    std::vector<uint32_t> held_codes;  // the blocks' cell codes with these cells marked held-out
    if (!c->dblocks_host.empty()) {
        held_mark = c->dmask_host;
        held_codes = c->dcodes_host;
    }
    for (int64_t e = 0; e < n; ++e) {
        c->ho_part[e] = part_of(c, row[e], col[e]);
        const int32_t db = c->dblock_of.empty() ? -1
                                                : c->dblock_of[static_cast<size_t>(c->row_piece[row[e]]) * B + c->col_piece[col[e]]];
        if (db >= 0) {
            const DenseBlock &blk = c->dblocks_host[db];
            const int32_t i = row[e] - blk.row0, j = col[e] - blk.col0;
            const size_t cell = static_cast<size_t>(blk.v_off) + static_cast<size_t>(i) * blk.ld + j;
            if (c->dmask_host[cell] == kMaskTrain) return c->fail(PSGLD_E_STATE, "held-out cell is also a training entry");
            if (held_mark[cell] == kMaskHeld) return c->fail(PSGLD_E_ARG, "duplicate held-out cell");
            held_mark[cell] = kMaskHeld;
            held_codes[cell / 16] |= uint32_t{kMaskHeld} << (2 * (cell % 16));
            in_dense[e] = 1;
            const int32_t wg_cols = kDenseTileCols * blk.n_sub;
            dh[c->dblock_first_tile[db] + j / wg_cols].push_back(DenseHeld{i, j % wg_cols, static_cast<int32_t>(e), 0});
            continue;
        }
        pre[static_cast<size_t>(c->ho_part[e]) * I + row[e] + 1]++;
    }
    for (size_t k = 1; k < pre.size(); ++k) pre[k] += pre[k - 1];
    std::vector<HeldEntry> he(n);
    {
        std::vector<int32_t> fill(pre.begin(), pre.end() - 1);
        for (int64_t e = 0; e < n; ++e)
            if (!in_dense[e])
                he[fill[static_cast<size_t>(c->ho_part[e]) * I + row[e]]++] =
                    HeldEntry{col[e] * c->Kp, static_cast<int32_t>(e)};
        he.resize(pre.back());
    }
    // dense-block cells, grouped by work-group, each group in column order
    std::vector<DenseHeld> dflat;
    for (size_t w = 0; w < dh.size(); ++w) {
        std::sort(dh[w].begin(), dh[w].end(), [](const DenseHeld &a, const DenseHeld &b) {
            return a.col != b.col ? a.col < b.col : a.row < b.row;
        });
        const int32_t first = static_cast<int32_t>(dflat.size());
        for (int sub = 0; sub <= kDenseSubTiles; ++sub)
            c->dtiles_host[w].ho[sub] =
                first + static_cast<int32_t>(std::lower_bound(dh[w].begin(), dh[w].end(), sub * kDenseTileCols,
                                                              [](const DenseHeld &h, int32_t col) { return h.col < col; }) -
                                             dh[w].begin());
        dflat.insert(dflat.end(), dh[w].begin(), dh[w].end());
    }
    if (!c->dblocks_host.empty()) {
        HIPTRY(c, hipMemcpy(c->dtiles, c->dtiles_host.data(), c->dtiles_host.size() * sizeof(DenseTile),
                            hipMemcpyHostToDevice));
        HIPTRY(c, hipMemcpy(c->dmask, held_codes.data(), held_codes.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    }
    // coordinate-block cells: distinct, and disjoint from the training entries
    std::vector<int32_t> rp(static_cast<size_t>(B) * I + 1);
    HIPTRY(c, hipMemcpy(rp.data(), c->rowptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<Entry> er(static_cast<size_t>(c->nnz_sparse));
    if (c->nnz_sparse) HIPTRY(c, hipMemcpy(er.data(), c->ent_r, er.size() * sizeof(Entry), hipMemcpyDeviceToHost));
    for (size_t k = 0; k + 1 < pre.size(); ++k) {
        std::sort(he.begin() + pre[k], he.begin() + pre[k + 1],
                  [](const HeldEntry &a, const HeldEntry &b) { return a.off < b.off; });
        for (int32_t m = pre[k]; m < pre[k + 1]; ++m) {
            if (m > pre[k] && he[m].off == he[m - 1].off) return c->fail(PSGLD_E_ARG, "duplicate held-out cell");
            const Entry *b0 = er.data() + rp[k], *b1 = er.data() + rp[k + 1];
            const Entry *f = std::lower_bound(b0, b1, he[m].off, [](const Entry &a, int32_t v) { return a.off < v; });
            if (f != b1 && f->off == he[m].off)
                return c->fail(PSGLD_E_STATE, "held-out cell is also a training entry");
        }
    }
    // the FP64 sums are kept in the order the kernels visit the cells --
    // coordinate cells by (part, row, column), then dense cells by tile -- so
    // the sums of one part are one contiguous range; ho_slot maps the
    // caller's order to it
    c->ho_slot.assign(static_cast<size_t>(n), -1);
    for (size_t m = 0; m < he.size(); ++m) {
        c->ho_slot[he[m].slot] = static_cast<int32_t>(m);
        he[m].slot = static_cast<int32_t>(m);
    }
    for (size_t m = 0; m < dflat.size(); ++m) {
        const int32_t slot = static_cast<int32_t>(he.size() + m);
        c->ho_slot[dflat[m].slot] = slot;
        dflat[m].slot = slot;
    }
    if ((s = upload(c, &c->ho_ptr, pre))) return s;
    if ((s = upload(c, &c->ho_ent, he))) return s;
    if ((s = upload(c, &c->dheld, dflat))) return s;
    if ((s = dev_alloc(c, &c->ho_sum, static_cast<size_t>(n)))) return s;
    HIPTRY(c, hipMemset(c->ho_sum, 0, std::max<int64_t>(n, 1) * sizeof(double)));
    c->n_ho = n;
    c->ho_has_val = val != nullptr;
    c->ho_val.assign(val ? val : nullptr, val ? val + n : nullptr);
    c->heldout_loaded = true;
    return PSGLD_OK;
}

psgld_status psgld_set_factors(psgld_ctx *c, const float *W, const float *H)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->loaded) return c->fail(PSGLD_E_STATE, "load data first");
    if (!W || !H) return c->fail(PSGLD_E_ARG, "W and H are required");
    const int64_t I = c->I, J = c->J;
    const int32_t K = c->K, Kp = c->Kp;
    std::vector<float> w(static_cast<size_t>(I) * Kp, 0.f), h(static_cast<size_t>(J) * Kp, 0.f);
    for (int64_t i = 0; i < I; ++i)
        for (int32_t k = 0; k < K; ++k) {
            float v = W[static_cast<size_t>(i) * K + k];
            if (!std::isfinite(v)) return c->fail(PSGLD_E_ARG, "non-finite W");
            w[static_cast<size_t>(i) * Kp + k] = c->prior.mirror ? std::fabs(v) : v;
        }
    for (int32_t k = 0; k < K; ++k)
        for (int64_t j = 0; j < J; ++j) {
            float v = H[static_cast<size_t>(k) * J + j];
            if (!std::isfinite(v)) return c->fail(PSGLD_E_ARG, "non-finite H");
            h[static_cast<size_t>(j) * Kp + k] = c->prior.mirror ? std::fabs(v) : v;
        }
    HIPTRY(c, use_device(c->opt.device));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    HIPTRY(c, hipMemcpy(c->W[c->cur], w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice));
    HIPTRY(c, hipMemcpy(c->H[c->cur], h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    c->factors_set = true;
    return PSGLD_OK;
}

psgld_status psgld_step(psgld_ctx *c, int64_t n_iter, const psgld_eps_schedule *sched)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    psgld_status s = check_schedule(c, sched);
    if (s) return s;
    if (n_iter < 0) return c->fail(PSGLD_E_ARG, "n_iter must be >= 0");
    if (!c->loaded || !c->factors_set) return c->fail(PSGLD_E_STATE, "load data and set factors first");
    if (c->t + n_iter >= INT32_MAX) return c->fail(PSGLD_E_ARG, "iteration counter would exceed 2^31");
    if (n_iter == 0) return PSGLD_OK;
    HIPTRY(c, use_device(c->opt.device));
    if ((s = ensure_eps_table(c, sched, c->t, c->t + n_iter))) return s;
    if (c->opt.persistent && c->dblocks_host.empty()) {
        psgld_ctx *one[1] = {c};
        return step_persistent(one, 1, n_iter, c->stream);
    }
    const int64_t L = graph_length(c);
    while (n_iter > 0) {
        if (L > 0 && n_iter >= L) {
            hipGraphExec_t exec;
            if ((s = get_graph(c, static_cast<int32_t>(c->t % c->B), c->cur, L, &exec))) return s;
            if (c->clock_host != c->t) {
                HIPTRY(c, launch_set_clock(c->clock, static_cast<int32_t>(c->t), c->stream));
                c->clock_host = c->t;
            }
            HIPTRY(c, hipGraphLaunch(exec, c->stream));
            c->clock_host += L;
            for (int64_t k = 0; k < L; ++k) account_iteration(c, c->t + k);
            c->cur ^= static_cast<int>(L & 1);
            c->t += L;
            n_iter -= L;
        } else {
            HIPTRY(c, enqueue_iteration(c, part_at(c, c->t), c->cur, nullptr,
                                        static_cast<int32_t>(c->t), true, c->stream));
            account_iteration(c, c->t);
            c->cur ^= 1;
            c->t += 1;
            n_iter -= 1;
        }
    }
    return PSGLD_OK;
}

}  // extern "C"

// ---- allocation-free stepping (psgld_step_static) -------------------------
namespace {
constexpr size_t kScratchBytes = size_t{16} << 20;
}  // namespace

// Scratch of psgld_step_static, one copy per device for the life of the
// process: the arrival counters of items cut over several work-groups, the
// step-size window of one call, and the partial gradients of the shares.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr size_t kScratchCounters = size_t{1} << 16;                  // int32 at byte 0
constexpr size_t kScratchEpsOffset = kScratchCounters * sizeof(int32_t);
constexpr size_t kScratchEps = size_t{1} << 16;                       // float2: iterations per call
constexpr size_t kScratchPartialOffset = kScratchEpsOffset + kScratchEps * sizeof(float2);
constexpr size_t kScratchPartialFloats = (kScratchBytes - kScratchPartialOffset) / sizeof(float);
static_assert(kScratchPartialOffset % 256 == 0, "scratch regions stay 256-byte aligned");

std::mutex g_scratch_mutex;
std::map<int, unsigned char *> g_scratch_addr;   // device -> device address of its `scratch`
float2 g_static_eps[kScratchEps];                // host staging of one call's step sizes (under the mutex)

// The device address of `scratch` on the current device `dev`.  The name
// itself is a host-side stand-in; only this address may be used from host
// code.  Looked up once per device.
psgld_status scratch_address(psgld_ctx *c, int dev, unsigned char **out)
{
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return c->fail(PSGLD_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_scratch_addr.emplace(dev, static_cast<unsigned char *>(ptr)).first;
    }
    *out = it->second;
    return PSGLD_OK;
}

}  // namespace

extern "C" {

psgld_status psgld_step_static(psgld_ctx *c, int64_t n_iter, const psgld_eps_schedule *sched)
{
    if (!c) return PSGLD_E_ARG;
    psgld_status s = check_schedule(c, sched);
    if (s) return s;
    if (n_iter < 0 || n_iter > static_cast<int64_t>(kScratchEps))
        return c->fail(PSGLD_E_ARG, "n_iter must be in [0, 65536]");
    if (!c->loaded || !c->factors_set) return c->fail(PSGLD_E_STATE, "load data and set factors first");
    if (c->t + n_iter >= INT32_MAX) return c->fail(PSGLD_E_ARG, "iteration counter would exceed 2^31");
    if (!c->dblocks_host.empty())
        return c->fail(PSGLD_E_UNSUPPORTED, "psgld_step_static runs coordinate-stored blocks only");
    if (static_cast<size_t>(c->max_splits) > kScratchCounters ||
        static_cast<size_t>(c->max_splits) * c->Kp > kScratchPartialFloats)
        return c->fail(PSGLD_E_UNSUPPORTED, "the schedule's split shares need more than the 16 MiB of static scratch");
    if (n_iter == 0) return PSGLD_OK;
    HIPTRY(c, use_device(c->opt.device));
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    unsigned char *base = nullptr;
    if ((s = scratch_address(c, c->opt.device, &base))) return s;
    int32_t *counters = reinterpret_cast<int32_t *>(base);
    float2 *eps_dev = reinterpret_cast<float2 *>(base + kScratchEpsOffset);
    float *partials = reinterpret_cast<float *>(base + kScratchPartialOffset);
    // the step sizes of t .. t + n_iter - 1, computed as psgld_step computes
    // them; this context's earlier work may still read the window
    const int64_t t0 = c->t;
    for (int64_t k = 0; k < n_iter; ++k) {
        const double eps = sched->a * std::pow(sched->t0 + static_cast<double>(t0 + k), -sched->gamma);
        g_static_eps[k] = make_float2(static_cast<float>(eps), static_cast<float>(std::sqrt(2.0 * eps)));
    }
    HIPTRY(c, hipStreamSynchronize(c->stream));
    HIPTRY(c, hipMemcpy(eps_dev, g_static_eps, static_cast<size_t>(n_iter) * sizeof(float2), hipMemcpyHostToDevice));
    // arrival counters start at zero (the kernels leave them at zero, but the
    // array is shared with every other call on this device)
    HIPTRY(c, launch_fill_i32(counters, 0, std::max<int32_t>(c->max_splits, 1), c->stream));
    const IterBuffers buf{eps_dev - t0, partials, counters};
    for (int64_t k = 0; k < n_iter; ++k) {
        HIPTRY(c, enqueue_iteration(c, part_at(c, c->t), c->cur, nullptr, static_cast<int32_t>(c->t), true,
                                    c->stream, &buf));
        account_iteration(c, c->t);
        c->cur ^= 1;
        c->t += 1;
    }
    return PSGLD_OK;
}

namespace {

// Auxiliary streams of a device for the kernel variants of a batched step,
// with their fork and join events: created on first use and kept for the
// life of the process (a stream costs about a millisecond to create).
// Default priority, like every stream here.  Callers hold g_aux_mutex while
// they enqueue on them.
constexpr int kAuxStreams = 8;
struct AuxStreams {
    hipStream_t s[kAuxStreams] = {};
    hipEvent_t join[kAuxStreams] = {};
    hipEvent_t fork = nullptr;
};
std::mutex g_aux_mutex;
std::map<int, AuxStreams> g_aux;

psgld_status aux_streams(psgld_ctx *c, AuxStreams **out)
{
    auto it = g_aux.find(c->opt.device);
    if (it == g_aux.end()) {
        AuxStreams a;
        HIPTRY(c, hipEventCreateWithFlags(&a.fork, hipEventDisableTiming));
        for (int i = 0; i < kAuxStreams; ++i) {
            HIPTRY(c, hipStreamCreateWithFlags(&a.s[i], hipStreamNonBlocking));
            HIPTRY(c, hipEventCreateWithFlags(&a.join[i], hipEventDisableTiming));
        }
        it = g_aux.emplace(c->opt.device, a).first;
    }
    *out = &it->second;
    return PSGLD_OK;
}

}  // namespace

psgld_status psgld_step_batch(psgld_ctx *const *ctxs, int32_t n, const int64_t *n_iter,
                              const psgld_eps_schedule *scheds)
{
    if (n < 0 || (n > 0 && (!ctxs || !n_iter || !scheds))) return PSGLD_E_ARG;
    if (n == 0) return PSGLD_OK;
    for (int32_t j = 0; j < n; ++j) {
        if (!ctxs[j]) return PSGLD_E_ARG;
        for (int32_t m = 0; m < j; ++m)
            if (ctxs[m] == ctxs[j]) return ctxs[j]->fail(PSGLD_E_ARG, "a context appears twice in the batch");
    }
    psgld_ctx *c0 = ctxs[0];
    int64_t max_n = 0;
    for (int32_t j = 0; j < n; ++j) {
        psgld_ctx *c = ctxs[j];
        c->err.clear();
        psgld_status s = check_schedule(c, &scheds[j]);
        if (s) return s;
        if (n_iter[j] < 0) return c->fail(PSGLD_E_ARG, "n_iter must be >= 0");
        if (!c->loaded || !c->factors_set) return c->fail(PSGLD_E_STATE, "load data and set factors first");
        if (c->t + n_iter[j] >= INT32_MAX) return c->fail(PSGLD_E_ARG, "iteration counter would exceed 2^31");
        if (c->opt.device != c0->opt.device || c->stream != c0->stream)
            return c->fail(PSGLD_E_ARG, "batched contexts must share one device and one stream");
        max_n = std::max(max_n, n_iter[j]);
    }
    HIPTRY(c0, use_device(c0->opt.device));
    hipStream_t stream = c0->stream;
    std::vector<char> batched(n, 0);
    for (int32_t j = 0; j < n; ++j) {
        psgld_ctx *c = ctxs[j];
        if (n_iter[j] == 0) continue;
        psgld_status s = ensure_eps_table(c, &scheds[j], c->t, c->t + n_iter[j]);
        if (s) return s;
        batched[j] = c->dblocks_host.empty() ? 1 : 0;
        if (!batched[j]) continue;
        if ((s = sync_job_desc(c))) return s;
        if (c->clock_host != c->t) {
            HIPTRY(c, launch_set_clock(c->clock, static_cast<int32_t>(c->t), stream));
            c->clock_host = c->t;
        }
    }
    bool persistent = false;
    for (int32_t j = 0; j < n; ++j)
        if (batched[j]) persistent = true;
    for (int32_t j = 0; j < n; ++j)
        if (batched[j] && !ctxs[j]->opt.persistent) persistent = false;
    if (persistent) {
        // one cooperative launch per (variant, iteration count) group
        std::map<std::tuple<int, int, int, int64_t>, std::vector<psgld_ctx *>> groups;
        for (int32_t j = 0; j < n; ++j)
            if (batched[j])
                groups[std::make_tuple(ctxs[j]->lpg, ctxs[j]->qpl, ctxs[j]->lik_kind, n_iter[j])].push_back(ctxs[j]);
        for (auto &g : groups) {
            psgld_status s = step_persistent(g.second.data(), static_cast<int>(g.second.size()), std::get<3>(g.first),
                                             stream);
            if (s) return s;
        }
        for (int32_t j = 0; j < n; ++j) {
            psgld_ctx *c = ctxs[j];
            if (batched[j] || n_iter[j] == 0) continue;
            for (int64_t k = 0; k < n_iter[j]; ++k) {
                HIPTRY(c, enqueue_iteration(c, part_at(c, c->t), c->cur, nullptr,
                                            static_cast<int32_t>(c->t), true, stream));
                account_iteration(c, c->t);
                c->cur ^= 1;
                c->t += 1;
            }
        }
        return PSGLD_OK;
    }
    // the batched contexts' clocks stay put during the call (launch k runs
    // iteration clock + k) and advance once at its end
    std::vector<int32_t *> clocks;
    std::vector<int32_t> deltas;
    std::map<std::tuple<int, int, int>, int> variant;   // kernel variant -> its stream slot
    for (int32_t j = 0; j < n; ++j)
        if (batched[j]) {
            clocks.push_back(ctxs[j]->clock);
            deltas.push_back(static_cast<int32_t>(n_iter[j]));
            variant.emplace(std::make_tuple(ctxs[j]->lpg, ctxs[j]->qpl, ctxs[j]->lik_kind), 0);
        }
    // Variants touch disjoint contexts, so with more than one each runs on an
    // auxiliary stream of its own (forked from and joined back into the
    // contexts' stream), and the small launches of different variants overlap
    // on the device instead of queueing behind each other.
    std::unique_lock<std::mutex> aux_lock;
    AuxStreams *aux = nullptr;
    int n_aux = 0;
    if (variant.size() > 1) {
        aux_lock = std::unique_lock<std::mutex>(g_aux_mutex);
        psgld_status s = aux_streams(c0, &aux);
        if (s) return s;
        n_aux = static_cast<int>(std::min<size_t>(variant.size(), kAuxStreams));
        int slot = 0;
        for (auto &v : variant) v.second = slot++ % n_aux;
        HIPTRY(c0, hipEventRecord(aux->fork, stream));
        for (int a = 0; a < n_aux; ++a) HIPTRY(c0, hipStreamWaitEvent(aux->s[a], aux->fork, 0));
    }
    for (int64_t k = 0; k < max_n; ++k) {
        // one launch per kernel variant (lanes per group, quads per lane,
        // likelihood) and 64 contexts
        std::map<std::tuple<int, int, int>, std::vector<int32_t>> groups;
        for (int32_t j = 0; j < n; ++j)
            if (k < n_iter[j] && batched[j])
                groups[std::make_tuple(ctxs[j]->lpg, ctxs[j]->qpl, ctxs[j]->lik_kind)].push_back(j);
        for (auto &g : groups) {
            const std::vector<int32_t> &js = g.second;
            const hipStream_t gs = aux ? aux->s[variant.at(g.first)] : stream;
            for (size_t first = 0; first < js.size(); first += kMaxBatch) {
                BatchArgs b{};
                b.k = static_cast<int32_t>(k);
                b.n = static_cast<int32_t>(std::min<size_t>(kMaxBatch, js.size() - first));
                b.wg_first[0] = 0;
                for (int32_t q = 0; q < b.n; ++q) {
                    psgld_ctx *c = ctxs[js[first + q]];
                    b.jobs[q] = c->job_desc;
                    b.wg_first[q + 1] = b.wg_first[q] + c->max_tasks;
                }
                HIPTRY(c0, launch_sparse_batch(b, std::get<2>(g.first), std::get<0>(g.first), std::get<1>(g.first), gs));
            }
        }
        for (int32_t j = 0; j < n; ++j) {
            if (k >= n_iter[j]) continue;
            psgld_ctx *c = ctxs[j];
            if (!batched[j])
                HIPTRY(c, enqueue_iteration(c, part_at(c, c->t), c->cur, nullptr,
                                            static_cast<int32_t>(c->t), true, stream));
            account_iteration(c, c->t);
            c->cur ^= 1;
            c->t += 1;
        }
    }
    for (int a = 0; a < n_aux; ++a) {
        HIPTRY(c0, hipEventRecord(aux->join[a], aux->s[a]));
        HIPTRY(c0, hipStreamWaitEvent(stream, aux->join[a], 0));
    }
    if (!clocks.empty())
        HIPTRY(c0, launch_advance_clocks(clocks.data(), deltas.data(), static_cast<int>(clocks.size()), stream));
    for (int32_t j = 0; j < n; ++j)
        if (batched[j]) ctxs[j]->clock_host = ctxs[j]->t;
    return PSGLD_OK;
}

psgld_status psgld_tune(psgld_ctx *c, const int32_t *candidates, int32_t n, int32_t iters,
                        const psgld_eps_schedule *sched, int32_t *chosen)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->loaded || !c->factors_set) return c->fail(PSGLD_E_STATE, "load data and set factors first");
    if (n < 1 || !candidates) return c->fail(PSGLD_E_ARG, "at least one candidate is required");
    for (int32_t k = 0; k < n; ++k)
        if (candidates[k] < 1) return c->fail(PSGLD_E_ARG, "candidates must be >= 1");
    psgld_status s;
    HIPTRY(c, use_device(c->opt.device));
    TuneChoice best{candidates[0], c->qpl};
    if (n > 1) {
        if ((s = check_schedule(c, sched))) return s;
        if ((s = sync_and_check(c))) return s;
        if (iters < 1) iters = c->B;
        if ((s = ensure_eps_table(c, sched, c->t, c->t + iters))) return s;
        // kernel variants: quads per lane 1, 2 or 4 with the lanes that cover
        // the row, where such a kernel is built
        std::vector<int> qpls;
        for (int q : {1, 2, 4})
            if (sparse_variant_exists(sparse_lanes_for(c->K, q), q)) qpls.push_back(q);
        // trials run on copies of the state, from the context's current t
        const size_t nw = static_cast<size_t>(c->I) * c->Kp + kFactorPad, nh = static_cast<size_t>(c->J) * c->Kp + kFactorPad;
        const int cur0 = c->cur;
        float *w0 = nullptr, *h0 = nullptr;
        if ((s = dev_alloc(c, &w0, nw)) || (s = dev_alloc(c, &h0, nh))) return s;
        HIPTRY(c, hipMemcpyAsync(w0, c->W[cur0], nw * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        HIPTRY(c, hipMemcpyAsync(h0, c->H[cur0], nh * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        hipEvent_t e0, e1;
        HIPTRY(c, hipEventCreate(&e0));
        HIPTRY(c, hipEventCreate(&e1));
        float best_ms = 0.f;
        bool first = true;
        for (int q : qpls)
            for (int32_t k = 0; k < n; ++k) {
                set_variant(c, q);
                c->sched.entries_per_group = candidates[k];
                if ((s = upload_schedule(c))) return s;
                float ms = 0.f;
                for (int rep = 0; rep < 2; ++rep) {   // first pass warms up
                    HIPTRY(c, hipMemcpyAsync(c->W[cur0], w0, nw * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
                    HIPTRY(c, hipMemcpyAsync(c->H[cur0], h0, nh * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
                    c->cur = cur0;
                    HIPTRY(c, hipEventRecord(e0, c->stream));
                    for (int32_t it = 0; it < iters; ++it)
                        HIPTRY(c, enqueue_iteration(c, part_at(c, c->t + it), (cur0 + it) & 1,
                                                    nullptr, static_cast<int32_t>(c->t + it), false, c->stream));
                    HIPTRY(c, hipEventRecord(e1, c->stream));
                    HIPTRY(c, hipEventSynchronize(e1));
                    HIPTRY(c, hipEventElapsedTime(&ms, e0, e1));
                }
                if (first || ms < best_ms) {
                    best_ms = ms;
                    best = TuneChoice{candidates[k], q};
                    first = false;
                }
            }
        HIPTRY(c, hipMemcpyAsync(c->W[cur0], w0, nw * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        HIPTRY(c, hipMemcpyAsync(c->H[cur0], h0, nh * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        c->cur = cur0;
        HIPTRY(c, hipStreamSynchronize(c->stream));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        dev_free(c, w0);
        dev_free(c, h0);
        remember_choice(c, best);
    }
    set_variant(c, best.qpl);
    c->sched.entries_per_group = best.entries_per_group;
    if ((s = upload_schedule(c))) return s;
    if (chosen) *chosen = best.entries_per_group;
    return PSGLD_OK;
}

psgld_status psgld_set_schedule(psgld_ctx *c, int32_t entries_per_group, int32_t quads_per_lane)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->loaded) return c->fail(PSGLD_E_STATE, "load data first");
    if (entries_per_group < 1) return c->fail(PSGLD_E_ARG, "entries_per_group must be >= 1");
    if (quads_per_lane == 0) quads_per_lane = sparse_quads_per_lane(c->K);
    if (!sparse_variant_exists(sparse_lanes_for(c->K, quads_per_lane), quads_per_lane))
        return c->fail(PSGLD_E_ARG, "no kernel variant with that many quads per lane for this rank");
    HIPTRY(c, use_device(c->opt.device));
    set_variant(c, quads_per_lane);
    c->sched.entries_per_group = entries_per_group;
    return upload_schedule(c);
}

psgld_status psgld_schedule_info(psgld_ctx *c, int32_t *entries_per_group, int32_t *quads_per_lane,
                                 int32_t *lanes_per_group)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (entries_per_group) *entries_per_group = c->sched.entries_per_group;
    if (quads_per_lane) *quads_per_lane = c->qpl;
    if (lanes_per_group) *lanes_per_group = c->lpg;
    return PSGLD_OK;
}

psgld_status psgld_sync(psgld_ctx *c)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    return sync_and_check(c);
}

psgld_status psgld_get_factors(psgld_ctx *c, float *W, float *H)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->factors_set) return c->fail(PSGLD_E_STATE, "factors not set");
    if (!W || !H) return c->fail(PSGLD_E_ARG, "W and H are required");
    psgld_status s = sync_and_check(c);
    if (s && s != PSGLD_E_NUMERIC) return s;
    psgld_status s2;
    if ((s2 = fetch_factor(c, c->W[c->cur], c->I, false, W, 1.0))) return s2;
    if ((s2 = fetch_factor(c, c->H[c->cur], c->J, true, H, 1.0))) return s2;
    return s;
}

psgld_status psgld_num_samples(psgld_ctx *c, int64_t *S)
{
    if (!c || !S) return PSGLD_E_ARG;
    *S = c->n_kept;
    return PSGLD_OK;
}

psgld_status psgld_posterior_mean(psgld_ctx *c, double *W, double *H)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!W || !H) return c->fail(PSGLD_E_ARG, "W and H are required");
    if (c->n_kept == 0) return c->fail(PSGLD_E_STATE, "no samples kept yet");
    psgld_status s = sync_and_check(c);
    if (s) return s;
    const double inv = 1.0 / static_cast<double>(c->n_kept);
    if ((s = fetch_factor(c, c->sum[0], c->I, false, W, inv))) return s;
    return fetch_factor(c, c->sum[1], c->J, true, H, inv);
}

psgld_status psgld_posterior_var(psgld_ctx *c, double *W, double *H)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!W || !H) return c->fail(PSGLD_E_ARG, "W and H are required");
    if (c->n_kept == 0) return c->fail(PSGLD_E_STATE, "no samples kept yet");
    psgld_status s = sync_and_check(c);
    if (s) return s;
    const double inv = 1.0 / static_cast<double>(c->n_kept);
    const size_t nw = static_cast<size_t>(c->I) * c->K, nh = static_cast<size_t>(c->J) * c->K;
    std::vector<double> mw(nw), mh(nh);
    if ((s = fetch_factor(c, c->sum[0], c->I, false, mw.data(), inv))) return s;
    if ((s = fetch_factor(c, c->sum[1], c->J, true, mh.data(), inv))) return s;
    if ((s = fetch_factor(c, c->sum2[0], c->I, false, W, inv))) return s;
    if ((s = fetch_factor(c, c->sum2[1], c->J, true, H, inv))) return s;
    for (size_t m = 0; m < nw; ++m) W[m] -= mw[m] * mw[m];
    for (size_t m = 0; m < nh; ++m) H[m] -= mh[m] * mh[m];
    return PSGLD_OK;
}

psgld_status psgld_heldout_predictions(psgld_ctx *c, double *pred)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->heldout_loaded) return c->fail(PSGLD_E_STATE, "no held-out cells loaded");
    if (!pred && c->n_ho > 0) return c->fail(PSGLD_E_ARG, "pred is required");
    psgld_status s = sync_and_check(c);
    if (s) return s;
    std::vector<double> sums(static_cast<size_t>(c->n_ho));
    if (c->n_ho) HIPTRY(c, hipMemcpy(sums.data(), c->ho_sum, sums.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < c->n_ho; ++e) {
        const int64_t v = c->part_visits[c->ho_part[e]];
        pred[e] = v > 0 ? sums[c->ho_slot[e]] / static_cast<double>(v) : NAN;
    }
    return PSGLD_OK;
}

psgld_status psgld_heldout_rmse(psgld_ctx *c, double *rmse)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!rmse) return c->fail(PSGLD_E_ARG, "rmse is required");
    if (!c->heldout_loaded || !c->ho_has_val) return c->fail(PSGLD_E_STATE, "no held-out values loaded");
    std::vector<double> pred(static_cast<size_t>(c->n_ho));
    psgld_status s = psgld_heldout_predictions(c, pred.data());
    if (s) return s;
    double acc = 0.0;
    int64_t n = 0;
    for (int64_t e = 0; e < c->n_ho; ++e) {
        if (std::isnan(pred[e])) continue;
        const double d = static_cast<double>(c->ho_val[e]) - pred[e];
        acc += d * d;
        ++n;
    }
    if (n == 0) return c->fail(PSGLD_E_STATE, "no held-out cell visited after burn-in yet");
    *rmse = std::sqrt(acc / static_cast<double>(n));
    return PSGLD_OK;
}

psgld_status psgld_log_likelihood(psgld_ctx *c, double *ll)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!ll) return c->fail(PSGLD_E_ARG, "ll is required");
    if (!c->loaded || !c->factors_set) return c->fail(PSGLD_E_STATE, "load data and set factors first");
    HIPTRY(c, use_device(c->opt.device));
    HIPTRY(c, launch_loglik(c->W[c->cur], c->H[c->cur], c->row_of_entry, c->ent_r, c->nnz_sparse, c->K, c->Kp,
                            c->lik.beta, c->lik.phi, c->opt.mu_floor, c->ll_partials, c->ll_blocks, c->stream));
    const int nd = static_cast<int>(c->dblocks_host.size());
    HIPTRY(c, launch_dense_loglik(c->W[c->cur], c->H[c->cur], c->dblocks, nd, c->dval, c->dval16, c->dmask, c->K, c->Kp,
                                  c->lik.beta, c->lik.phi, c->opt.mu_floor, c->ll_partials + c->ll_blocks,
                                  kDenseLLPerBlock, c->stream));
    HIPTRY(c, launch_sum_in_order(c->ll_partials, c->ll_blocks + nd * kDenseLLPerBlock, c->ll_out, c->stream));
    psgld_status s = sync_and_check(c);
    if (s) return s;
    HIPTRY(c, hipMemcpy(ll, c->ll_out, sizeof(double), hipMemcpyDeviceToHost));
    return PSGLD_OK;
}

psgld_status psgld_iteration(psgld_ctx *c, int64_t *t)
{
    if (!c || !t) return PSGLD_E_ARG;
    *t = c->t;
    return PSGLD_OK;
}

psgld_status psgld_part_sizes(psgld_ctx *c, int64_t *n_p, int64_t *N)
{
    if (!c) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->loaded) return c->fail(PSGLD_E_STATE, "load data first");
    if (n_p)
        for (int32_t p = 0; p < c->B; ++p) n_p[p] = c->n_p[p];
    if (N) *N = c->N;
    return PSGLD_OK;
}

psgld_status psgld_get_state(psgld_ctx *c, void *buf, size_t *size)
{
    if (!c || !size) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->loaded || !c->factors_set) return c->fail(PSGLD_E_STATE, "load data and set factors first");
    const size_t nw = static_cast<size_t>(c->I) * c->Kp, nh = static_cast<size_t>(c->J) * c->Kp;
    const size_t need = 8 * sizeof(int64_t) + (nw + nh) * sizeof(float) + 2 * (nw + nh) * sizeof(double) +
                        static_cast<size_t>(c->n_ho) * sizeof(double) + static_cast<size_t>(c->B) * sizeof(int64_t);
    if (!buf) {
        *size = need;
        return PSGLD_OK;
    }
    if (*size < need) return c->fail(PSGLD_E_ARG, "state buffer too small");
    psgld_status s = sync_and_check(c);
    if (s) return s;
    char *p = static_cast<char *>(buf);
    const int64_t hdr[8] = {kStateMagic, kStateVersion, c->I, c->J, c->K, c->B, c->t, c->n_kept};
    std::memcpy(p, hdr, sizeof(hdr));
    p += sizeof(hdr);
    HIPTRY(c, hipMemcpy(p, c->W[c->cur], nw * sizeof(float), hipMemcpyDeviceToHost));
    p += nw * sizeof(float);
    HIPTRY(c, hipMemcpy(p, c->H[c->cur], nh * sizeof(float), hipMemcpyDeviceToHost));
    p += nh * sizeof(float);
    for (int side = 0; side < 2; ++side) {
        const size_t n = side == 0 ? nw : nh;
        HIPTRY(c, hipMemcpy(p, c->sum[side], n * sizeof(double), hipMemcpyDeviceToHost));
        p += n * sizeof(double);
        HIPTRY(c, hipMemcpy(p, c->sum2[side], n * sizeof(double), hipMemcpyDeviceToHost));
        p += n * sizeof(double);
    }
    if (c->n_ho) {
        // saved in the caller's order of the held-out cells
        std::vector<double> sums(static_cast<size_t>(c->n_ho));
        HIPTRY(c, hipMemcpy(sums.data(), c->ho_sum, sums.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int64_t e = 0; e < c->n_ho; ++e) std::memcpy(p + e * sizeof(double), &sums[c->ho_slot[e]], sizeof(double));
    }
    p += static_cast<size_t>(c->n_ho) * sizeof(double);
    std::memcpy(p, c->part_visits.data(), static_cast<size_t>(c->B) * sizeof(int64_t));
    *size = need;
    return PSGLD_OK;
}

psgld_status psgld_set_state(psgld_ctx *c, const void *buf, size_t size)
{
    if (!c || !buf) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->loaded) return c->fail(PSGLD_E_STATE, "load data first");
    const size_t nw = static_cast<size_t>(c->I) * c->Kp, nh = static_cast<size_t>(c->J) * c->Kp;
    const size_t need = 8 * sizeof(int64_t) + (nw + nh) * sizeof(float) + 2 * (nw + nh) * sizeof(double) +
                        static_cast<size_t>(c->n_ho) * sizeof(double) + static_cast<size_t>(c->B) * sizeof(int64_t);
    if (size != need) return c->fail(PSGLD_E_ARG, "state size does not match this context");
    const char *p = static_cast<const char *>(buf);
    int64_t hdr[8];
    std::memcpy(hdr, p, sizeof(hdr));
    p += sizeof(hdr);
    if (hdr[0] != kStateMagic || hdr[1] != kStateVersion || hdr[2] != c->I || hdr[3] != c->J ||
        hdr[4] != c->K || hdr[5] != c->B)
        return c->fail(PSGLD_E_ARG, "state was saved from a different problem");
    HIPTRY(c, use_device(c->opt.device));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    HIPTRY(c, hipMemcpy(c->W[c->cur], p, nw * sizeof(float), hipMemcpyHostToDevice));
    p += nw * sizeof(float);
    HIPTRY(c, hipMemcpy(c->H[c->cur], p, nh * sizeof(float), hipMemcpyHostToDevice));
    p += nh * sizeof(float);
    for (int side = 0; side < 2; ++side) {
        const size_t n = side == 0 ? nw : nh;
        HIPTRY(c, hipMemcpy(c->sum[side], p, n * sizeof(double), hipMemcpyHostToDevice));
        p += n * sizeof(double);
        HIPTRY(c, hipMemcpy(c->sum2[side], p, n * sizeof(double), hipMemcpyHostToDevice));
        p += n * sizeof(double);
    }
    if (c->n_ho) {
        std::vector<double> sums(static_cast<size_t>(c->n_ho));
        for (int64_t e = 0; e < c->n_ho; ++e) std::memcpy(&sums[c->ho_slot[e]], p + e * sizeof(double), sizeof(double));
        HIPTRY(c, hipMemcpy(c->ho_sum, sums.data(), sums.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    p += static_cast<size_t>(c->n_ho) * sizeof(double);
    std::memcpy(c->part_visits.data(), p, static_cast<size_t>(c->B) * sizeof(int64_t));
    c->t = hdr[6];
    c->n_kept = hdr[7];
    c->factors_set = true;
    return PSGLD_OK;
}

psgld_status psgld_memory_bytes(psgld_ctx *c, int64_t *bytes)
{
    if (!c || !bytes) return PSGLD_E_ARG;
    *bytes = c->bytes;
    return PSGLD_OK;
}

psgld_status psgld_get_stream(psgld_ctx *c, void **stream)
{
    if (!c || !stream) return PSGLD_E_ARG;
    c->err.clear();
    psgld_status s = ensure_device(c);
    if (s) return s;
    *stream = c->stream;
    return PSGLD_OK;
}

const char *psgld_last_error(const psgld_ctx *c)
{
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

void psgld_destroy(psgld_ctx *c)
{
    if (!c) return;
    if (c->device_ready) {
        (void)use_device(c->opt.device);
        (void)hipStreamSynchronize(c->stream);
        drop_graphs(c);
        for (auto &blk : c->allocs) release_block(c, blk.first, blk.second);
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
    }
    delete c;
}

psgld_status psgld_part_at(psgld_ctx *c, int64_t t, int32_t *part)
{
    if (!c || !part || t < 0) return PSGLD_E_ARG;
    c->err.clear();
    if (!c->loaded) return c->fail(PSGLD_E_STATE, "load data first");
    *part = part_at(c, t);
    return PSGLD_OK;
}

psgld_status psgld_balanced_pieces(int64_t n, const int64_t *weight, int32_t B, int32_t *piece)
{
    if (n < 1 || B < 1 || n < B || !weight || !piece) return PSGLD_E_ARG;
    for (int64_t m = 0; m < n; ++m)
        if (weight[m] < 0) return PSGLD_E_ARG;
    std::vector<int64_t> order(static_cast<size_t>(n));
    std::iota(order.begin(), order.end(), int64_t{0});
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return weight[a] > weight[b]; });
    // least-loaded piece first (lowest index on ties): a heap of (load, piece)
    std::vector<std::pair<int64_t, int32_t>> heap;
    for (int32_t b = 0; b < B; ++b) heap.emplace_back(0, b);
    auto later = [](const std::pair<int64_t, int32_t> &x, const std::pair<int64_t, int32_t> &y) { return x > y; };
    std::make_heap(heap.begin(), heap.end(), later);
    for (int64_t m : order) {
        std::pop_heap(heap.begin(), heap.end(), later);
        auto &top = heap.back();
        piece[m] = top.second;
        top.first += weight[m];
        std::push_heap(heap.begin(), heap.end(), later);
    }
    return PSGLD_OK;
}

psgld_status psgld_philox_blocks(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out,
                                 int32_t device)
{
    if (n < 0 || (n > 0 && (!ctr || !key || !out))) return PSGLD_E_ARG;
    if (n == 0) return PSGLD_OK;
    if (hipSetDevice(device) != hipSuccess || !is_gfx950(device)) return PSGLD_E_DEVICE;
    uint32_t *dc = nullptr, *dk = nullptr, *dout = nullptr;
    psgld_status s = PSGLD_OK;
    if (hipMalloc(&dc, n * 16) != hipSuccess || hipMalloc(&dk, n * 8) != hipSuccess ||
        hipMalloc(&dout, n * 16) != hipSuccess) {
        s = PSGLD_E_NOMEM;
    } else if (hipMemcpy(dc, ctr, n * 16, hipMemcpyHostToDevice) != hipSuccess ||
               hipMemcpy(dk, key, n * 8, hipMemcpyHostToDevice) != hipSuccess ||
               launch_philox_blocks(n, dc, dk, dout, nullptr) != hipSuccess ||
               hipMemcpy(out, dout, n * 16, hipMemcpyDeviceToHost) != hipSuccess) {
        s = PSGLD_E_DEVICE;
    }
    (void)hipFree(dc);
    (void)hipFree(dk);
    (void)hipFree(dout);
    return s;
}

psgld_status psgld_normals(int64_t n, uint64_t seed, const int64_t *t, const uint32_t *stream,
                           const int64_t *index, int32_t K, float *z, float *radius, int32_t device)
{
    if (n < 0 || K < 1 || (n > 0 && (!t || !stream || !index || !z || !radius))) return PSGLD_E_ARG;
    if (n == 0) return PSGLD_OK;
    if (hipSetDevice(device) != hipSuccess || !is_gfx950(device)) return PSGLD_E_DEVICE;
    int64_t *dt = nullptr, *di = nullptr;
    uint32_t *ds = nullptr;
    float *dz = nullptr, *dr = nullptr;
    psgld_status s = PSGLD_OK;
    const size_t nz = static_cast<size_t>(n) * K * sizeof(float);
    if (hipMalloc(&dt, n * 8) != hipSuccess || hipMalloc(&di, n * 8) != hipSuccess ||
        hipMalloc(&ds, n * 4) != hipSuccess || hipMalloc(&dz, nz) != hipSuccess ||
        hipMalloc(&dr, nz) != hipSuccess) {
        s = PSGLD_E_NOMEM;
    } else if (hipMemcpy(dt, t, n * 8, hipMemcpyHostToDevice) != hipSuccess ||
               hipMemcpy(di, index, n * 8, hipMemcpyHostToDevice) != hipSuccess ||
               hipMemcpy(ds, stream, n * 4, hipMemcpyHostToDevice) != hipSuccess ||
               launch_normals(n, seed, dt, ds, di, K, dz, dr, nullptr) != hipSuccess ||
               hipMemcpy(z, dz, nz, hipMemcpyDeviceToHost) != hipSuccess ||
               hipMemcpy(radius, dr, nz, hipMemcpyDeviceToHost) != hipSuccess) {
        s = PSGLD_E_DEVICE;
    }
    (void)hipFree(dt);
    (void)hipFree(di);
    (void)hipFree(ds);
    (void)hipFree(dz);
    (void)hipFree(dr);
    return s;
}

}  // extern "C"

// One PSGLD iteration over one part, for coordinate-stored blocks.
//
// Eq. (8)-(9) decompose the part's update into independent per-block updates;
// within a block, row i of W needs g_i = sum_j e_ij h_j over its entries and
// column j of H needs sum_i e_ij w_i, both at the previous state.  Each row
// of W and each column of H lies in exactly one block of the part
// (Definition 2), so one launch updates all of W and H:
//
//  * an "item" is a row of W (side 0) or a column of H (side 1);
//  * the part's entries are stored twice, row-sorted (for W items) and
//    column-sorted (for H items), so each item's gradient is a sequential
//    sum over a contiguous run of entries -- no atomics on values;
//  * a group of LPG lanes owns one item, each lane four consecutive k
//    (a float4), so a K-length dot product is four FMAs plus a log2(LPG)
//    step butterfly across the group (DPP inside 16-lane rows);
//  * long items are split over G groups of one work-group, combined in LDS
//    in a fixed order, and the longest over several work-groups, combined
//    in a fixed order by whichever share finishes last;
//  * the Langevin step, noise, prior and mirroring are applied by the item's
//    lead group right after its gradient, into the other ping-pong buffer;
//    the old buffers are only read, so no item waits for another.
#include <algorithm>

#include "internal.hpp"
#include "noise.hpp"

namespace psgld {
namespace {

constexpr int kBlockThreads = 256;

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over the LPG lanes of a group; every lane gets the same bits (each
// stage adds a symmetric pair of lanes).  xor 1 and xor 2 are quad
// permutations, then half-row and row mirrors pair the 4- and 8-lane halves
// of a 16-lane row; across rows a swizzle (xor 16) and a permute (xor 32).
template <int LPG>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (LPG >= 2) v += dpp<0xB1>(v);
    if constexpr (LPG >= 4) v += dpp<0x4E>(v);
    if constexpr (LPG >= 8) v += dpp<0x141>(v);
    if constexpr (LPG >= 16) v += dpp<0x140>(v);
    if constexpr (LPG >= 32) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
    if constexpr (LPG >= 64) v += __shfl_xor(v, 32);
    return v;
}

// The same butterfly applied to N independent values stage by stage, so
// consecutive DPP operations never depend on each other.
template <int LPG, int N>
__device__ __forceinline__ void group_sum_n(float (&v)[N])
{
#pragma unroll
    for (int n = 0; n < N; ++n)
        if constexpr (LPG >= 2) v[n] += dpp<0xB1>(v[n]);
#pragma unroll
    for (int n = 0; n < N; ++n)
        if constexpr (LPG >= 4) v[n] += dpp<0x4E>(v[n]);
#pragma unroll
    for (int n = 0; n < N; ++n)
        if constexpr (LPG >= 8) v[n] += dpp<0x141>(v[n]);
#pragma unroll
    for (int n = 0; n < N; ++n)
        if constexpr (LPG >= 16) v[n] += dpp<0x140>(v[n]);
#pragma unroll
    for (int n = 0; n < N; ++n)
        if constexpr (LPG >= 32) v[n] += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v[n]), 0x401F));
#pragma unroll
    for (int n = 0; n < N; ++n)
        if constexpr (LPG >= 64) v[n] += __shfl_xor(v[n], 32);
}

__device__ __forceinline__ float dot4(const float4 &a, const float4 &b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
}

__device__ __forceinline__ void axpy4(float4 &acc, float r, const float4 &o)
{
    acc.x += r * o.x;
    acc.y += r * o.y;
    acc.z += r * o.z;
    acc.w += r * o.w;
}

__device__ __forceinline__ void add4(float4 &acc, const float4 &o)
{
    acc.x += o.x;
    acc.y += o.y;
    acc.z += o.z;
    acc.w += o.w;
}

template <int LIK>
__device__ __forceinline__ float residual(float v, float mu, const SparseIterArgs &a)
{
    return tweedie_residual<LIK>(v, mu, a.inv_phi, a.beta, a.mu_floor);
}

__device__ __forceinline__ float4 load4(const float *p) { return *reinterpret_cast<const float4 *>(p); }

// The side's member of a W/H pair, by selection rather than indexing, so an
// argument block held in registers is never indexed dynamically.
template <typename T>
__device__ __forceinline__ T pick(int side, T w, T h)
{
    return side ? h : w;
}

// Entries per batch: a batch's partner loads are QPL float4 per lane each,
// so the batch holds 8 / QPL entries (32 partner registers either way).
template <int QPL>
constexpr int kBatch = 8 / QPL;

// Quad m of a lane: k = 4 (lane + m LPG) .. + 3, so consecutive lanes read
// consecutive 16-byte pieces of a row.
template <int LPG>
__device__ __forceinline__ int quad_of(int lane, int m)
{
    return lane + m * LPG;
}

// One group's view of its current item: the lane's quads of the item's own
// row (x), and the first batch of its entry records.
template <int QPL>
struct ItemStart {
    float4 x[QPL];
    Entry first[kBatch<QPL>];
};

template <int LPG, int QPL>
__device__ __forceinline__ ItemStart<QPL> start_item(const SparseIterArgs &a, const WgTask &task,
                                                     const GroupRec &rec, int lane)
{
    ItemStart<QPL> st;
    const float *row = pick(task.side, a.x_old[0], a.x_old[1]) + static_cast<size_t>(rec.item) * a.Kp;
#pragma unroll
    for (int m = 0; m < QPL; ++m) {
        const int q = quad_of<LPG>(lane, m);
        st.x[m] = (rec.item >= 0 && q < a.nq) ? load4(row + 4 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const Entry *ent = pick(task.side, a.ent[0], a.ent[1]);
    const int s0 = rec.item >= 0 ? rec.s0 : 0;
#pragma unroll
    for (int u = 0; u < kBatch<QPL>; ++u) st.first[u] = ent[s0 + u];
    return st;
}

// Gradient of the likelihood over the group's entries [s0, s1), in batches
// of kBatch entries whose records are in registers before the batch starts
// (the first batch from start_item, each next one fetched while the current
// one is reduced).  Quads past ceil(K/4) have x = 0 and read up to one row
// ahead (the factor arrays are padded and zero-initialised); a batch's
// records past s1 belong to the next item or to the padding of the entry
// array; in the last batch their partner rows are not loaded and their
// contributions are masked.  A short item is thus one round of partner loads.
template <int LPG, int QPL, int LIK>
__device__ __forceinline__ void item_gradient(const SparseIterArgs &a, const WgTask &task, const GroupRec &rec,
                                              const ItemStart<QPL> &st, int lane, float4 (&acc)[QPL])
{
    constexpr int U = kBatch<QPL>;
    const Entry *__restrict__ ent = pick(task.side, a.ent[0], a.ent[1]);
    const float *other_lane = pick(task.side, a.x_old[1], a.x_old[0]) + 4 * lane;
    const int s0 = rec.s0, s1 = rec.item >= 0 ? rec.s1 : rec.s0;
    const int full_end = s0 + (s1 - s0) / U * U;
#pragma unroll
    for (int m = 0; m < QPL; ++m) acc[m] = make_float4(0.f, 0.f, 0.f, 0.f);
    Entry cur[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = st.first[u];
    int e = s0;
    for (; e < full_end; e += U) {
        float4 o[U][QPL];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int m = 0; m < QPL; ++m) o[u][m] = load4(other_lane + cur[u].off + 4 * m * LPG);
        Entry nxt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) nxt[u] = ent[e + U + u];
        float mu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            mu[u] = dot4(st.x[0], o[u][0]);
#pragma unroll
            for (int m = 1; m < QPL; ++m) mu[u] += dot4(st.x[m], o[u][m]);
        }
        group_sum_n<LPG, U>(mu);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float r = residual<LIK>(cur[u].val, mu[u], a);
#pragma unroll
            for (int m = 0; m < QPL; ++m) axpy4(acc[m], r, o[u][m]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
    const int n = s1 - e;   // 0 .. U - 1 entries left
    if (n > 0) {
        // the records past s1 load no partner row (their lanes are masked
        // off), which spares the L2 the requests of short items
        float4 o[U][QPL];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int m = 0; m < QPL; ++m)
                o[u][m] = u < n ? load4(other_lane + cur[u].off + 4 * m * LPG) : make_float4(0.f, 0.f, 0.f, 0.f);
        float mu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            mu[u] = dot4(st.x[0], o[u][0]);
#pragma unroll
            for (int m = 1; m < QPL; ++m) mu[u] += dot4(st.x[m], o[u][m]);
        }
        group_sum_n<LPG, U>(mu);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (u < n) {
                const float r = residual<LIK>(cur[u].val, mu[u], a);
#pragma unroll
                for (int m = 0; m < QPL; ++m) axpy4(acc[m], r, o[u][m]);
            }
    }
}

// Held-out sums, then the Langevin step of the lane's quads with the full
// gradient g, by the item's lead group.
template <int LPG, int QPL>
__device__ __forceinline__ void item_update(const SparseIterArgs &a, const IterScalars &it, int side, int item,
                                            const float4 (&x)[QPL], const float4 (&g)[QPL], int lane)
{
    if (side == 0 && it.do_heldout) {
        // held-out cells of the row in this block, a batch at a time: the
        // batch's records, partner loads and FP64 sums are all in flight
        // together (records past the row's last cell are clamped to it and
        // their sums skipped)
        constexpr int U = kBatch<QPL>;
        const float *other_lane = a.x_old[1] + 4 * lane;
        const int hb = a.ho_ptr[item], he = a.ho_ptr[item + 1];
        for (int h0 = hb; h0 < he; h0 += U) {
            HeldEntry c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) c[u] = a.ho_ent[min(h0 + u, he - 1)];
            float mu[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                mu[u] = dot4(x[0], load4(other_lane + c[u].off));
#pragma unroll
                for (int m = 1; m < QPL; ++m) mu[u] += dot4(x[m], load4(other_lane + c[u].off + 4 * m * LPG));
            }
            group_sum_n<LPG, U>(mu);
            if (lane == 0) {
                double prev[U];
#pragma unroll
                for (int u = 0; u < U; ++u) prev[u] = h0 + u < he ? a.ho_sum[c[u].slot] : 0.0;
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (h0 + u < he) a.ho_sum[c[u].slot] = prev[u] + static_cast<double>(mu[u]);
            }
        }
    }
    const bool frozen = (a.flags & (side == 0 ? PSGLD_TEST_FREEZE_W : PSGLD_TEST_FREEZE_H)) != 0;
    const bool noisy = !frozen && !(a.flags & PSGLD_TEST_NOISE_OFF);
    const float lam = pick(side, a.lambda[0], a.lambda[1]);
    float *xnew = pick(side, a.x_new[0], a.x_new[1]);
    bool finite = true;
#pragma unroll
    for (int m = 0; m < QPL; ++m) {
        const int q = quad_of<LPG>(lane, m);
        if (q >= a.nq) {
            // padding of the row: rewritten as zeros, so the row's cache
            // lines are written whole
            if (4 * q < a.Kp)
                *reinterpret_cast<float4 *>(xnew + static_cast<size_t>(item) * a.Kp + 4 * q) =
                    make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        float z[4] = {0.f, 0.f, 0.f, 0.f};
        if (noisy) {
            const Normal4 nz = normal4(a.seed_lo, a.seed_hi, it.t, static_cast<uint32_t>(side),
                                       static_cast<uint32_t>(item), static_cast<uint32_t>(q));
            z[0] = nz.z[0];
            z[1] = nz.z[1];
            z[2] = nz.z[2];
            z[3] = nz.z[3];
        }
        const float xo[4] = {x[m].x, x[m].y, x[m].z, x[m].w};
        const float gr[4] = {g[m].x, g[m].y, g[m].z, g[m].w};
        float xn[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            float v = xo[c];
            if (!frozen) {
                const float pg = a.prior_kind == PSGLD_PRIOR_EXPONENTIAL ? (xo[c] >= 0.f ? -lam : lam)
                                                                         : -lam * xo[c];
                v = xo[c] + it.eps * (a.scale * gr[c] + pg) + it.sigma * z[c];
                if (a.mirror) v = fabsf(v);
            }
            if (4 * q + c >= a.K) v = 0.f;
            finite = finite && isfinite(v);
            xn[c] = v;
        }
        const size_t off = static_cast<size_t>(item) * a.Kp + 4 * q;
        *reinterpret_cast<float4 *>(xnew + off) = make_float4(xn[0], xn[1], xn[2], xn[3]);
        if (it.do_moments) {
            double2 *s = reinterpret_cast<double2 *>(pick(side, a.sum[0], a.sum[1]) + off);
            double2 *s2 = reinterpret_cast<double2 *>(pick(side, a.sum2[0], a.sum2[1]) + off);
            const double d0 = xn[0], d1 = xn[1], d2 = xn[2], d3 = xn[3];
            double2 p0 = s[0], p1 = s[1], q0 = s2[0], q1 = s2[1];
            p0.x += d0;
            p0.y += d1;
            p1.x += d2;
            p1.y += d3;
            q0.x += d0 * d0;
            q0.y += d1 * d1;
            q1.x += d2 * d2;
            q1.y += d3 * d3;
            s[0] = p0;
            s[1] = p1;
            s2[0] = q0;
            s2[1] = q1;
        }
    }
    if (!finite) atomicMin(a.nonfinite, static_cast<int32_t>(it.t));
}

// One work-group's task t of the part.  The task's records, then each
// group's own row and entries, then its partner rows are fetched; the item's
// lead group applies the update.
template <int LPG, int QPL, int LIK>
__device__ __forceinline__ void sparse_task(const SparseIterArgs &a, const IterScalars &it, int t)
{
    constexpr int Q = kBlockThreads / LPG;
    __shared__ float4 partial[QPL][kBlockThreads];
    __shared__ int is_last;
    const int tid = threadIdx.x;
    const int g = tid / LPG;
    const int lane = tid % LPG;
    const WgTask task = a.tasks[t];
    const GroupRec rec = a.recs[static_cast<size_t>(t) * Q + g];
    const ItemStart<QPL> st = start_item<LPG, QPL>(a, task, rec, lane);
    const int G = 1 << task.glog2;
    const int sub = g & (G - 1);
    float4 acc[QPL];
    item_gradient<LPG, QPL, LIK>(a, task, rec, st, lane, acc);

    // Items split over G groups: combine the partial sums in a fixed order.
    if (G > 1) {
#pragma unroll
        for (int m = 0; m < QPL; ++m) partial[m][tid] = acc[m];
        __syncthreads();
        if (sub == 0) {
#pragma unroll
            for (int m = 0; m < QPL; ++m) {
                acc[m] = make_float4(0.f, 0.f, 0.f, 0.f);
                for (int s = 0; s < G; ++s) add4(acc[m], partial[m][(g + s) * LPG + lane]);
            }
        }
    }
    // Items split over work-groups: publish this share; the last share to
    // arrive sums all shares in slot order.  Only the partials cross
    // work-groups, so instead of a release/acquire pair (an agent-scope
    // release writes back, and an acquire invalidates, the whole L2 of the
    // XCD, which would evict the partner rows other work-groups are
    // gathering) the ordering is made at the level of the gfx950 ISA:
    //  1. the partials are relaxed system-scope atomic stores, which compile
    //     to global_store_dword ... sc0 sc1: written through every cache
    //     level to memory;
    //  2. s_waitcnt vmcnt(0) holds the wave until each of those stores has
    //     been acknowledged at that scope, and the work-group barrier holds
    //     thread 0 until every wave has done so;
    //  3. only then does thread 0 count the arrival with an agent-scope
    //     atomic add (atomic across all XCDs of the device);
    //  4. the share that sees the count n_split - 1 reads every partial with
    //     relaxed system-scope loads (global_load_dword ... sc0 sc1: no cache
    //     level answers them), issued after the add has returned, since
    //     which share reads depends on the value it returned.
    // So every partial a last share reads was in memory before its writer's
    // arrival was counted.  This rests on the ISA's cache-bypass bits, not
    // on a happens-before edge of the HIP memory model.  Tested by stepping
    // Zipf(1.1)-skewed chains with items cut into dozens of shares and
    // comparing every single step with the FP64 oracle.
    bool lead = rec.item >= 0 && rec.lead;
    if (task.n_split > 0) {
        float *slot = a.split_partial + static_cast<size_t>(task.split_first + task.split_idx) * a.Kp;
        if (g == 0) {
#pragma unroll
            for (int m = 0; m < QPL; ++m) {
                const int q = quad_of<LPG>(lane, m);
                if (q >= a.nq) continue;
                __hip_atomic_store(slot + 4 * q + 0, acc[m].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(slot + 4 * q + 1, acc[m].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(slot + 4 * q + 2, acc[m].z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(slot + 4 * q + 3, acc[m].w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the stores are complete
        __syncthreads();
        if (tid == 0) {
            int32_t *cnt = a.split_count + task.split_first;
            const int old = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int last = old == task.n_split - 1;
            if (last) __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            is_last = last;
        }
        __syncthreads();
        if (is_last) {
            if (g == 0) {
                const float *first = a.split_partial + static_cast<size_t>(task.split_first) * a.Kp;
#pragma unroll
                for (int m = 0; m < QPL; ++m) {
                    const int q = quad_of<LPG>(lane, m);
                    acc[m] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (q >= a.nq) continue;
                    for (int s = 0; s < task.n_split; ++s) {
                        const float *pq = first + static_cast<size_t>(s) * a.Kp + 4 * q;
                        acc[m].x += __hip_atomic_load(pq + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        acc[m].y += __hip_atomic_load(pq + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        acc[m].z += __hip_atomic_load(pq + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        acc[m].w += __hip_atomic_load(pq + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    }
                }
            }
        } else {
            lead = false;
        }
    }

    if (lead) item_update<LPG, QPL>(a, it, task.side, rec.item, st.x, acc, lane);
}

// One work-group per task of the part.
template <int LPG, int QPL, int LIK>
__global__ __launch_bounds__(kBlockThreads) void sparse_iter_kernel(SparseIterArgs a)
{
    sparse_task<LPG, QPL, LIK>(a, iter_scalars(a.clk), blockIdx.x);
}

// Task `task` of context d at iteration t, with exactly the arguments a
// single-context launch would pass.  Returns without work when the current
// part has fewer tasks.
template <int LPG, int QPL, int LIK>
__device__ __forceinline__ void job_task(const JobDesc &d, int32_t t, int task)
{
    const int p = d.part_tab ? d.part_tab[t] : t % d.B;
    if (task >= d.n_tasks[p]) return;
    const int cur = (t + d.cur_phase) & 1;
    constexpr int Q = kBlockThreads / LPG;
    SparseIterArgs a;
    a.x_old[0] = d.W[cur];
    a.x_old[1] = d.H[cur];
    a.x_new[0] = d.W[cur ^ 1];
    a.x_new[1] = d.H[cur ^ 1];
    a.ptr[0] = d.rowptr + static_cast<size_t>(p) * d.I;
    a.ptr[1] = d.colptr + static_cast<size_t>(p) * d.J;
    a.ent[0] = d.ent[0];
    a.ent[1] = d.ent[1];
    a.tasks = d.tasks + d.task_off[p];
    a.recs = d.recs + static_cast<size_t>(d.task_off[p]) * Q;
    a.n_tasks = d.n_tasks[p];
    a.split_partial = d.split_partial;
    a.split_count = d.split_count;
    a.K = d.K;
    a.Kp = d.Kp;
    a.nq = d.nq;
    a.scale = d.scale[p];
    a.lambda[0] = d.lambda[0];
    a.lambda[1] = d.lambda[1];
    a.inv_phi = d.inv_phi;
    a.beta = d.beta;
    a.mu_floor = d.mu_floor;
    a.seed_lo = d.seed_lo;
    a.seed_hi = d.seed_hi;
    a.mirror = d.mirror;
    a.prior_kind = d.prior_kind;
    a.flags = d.flags;
    a.clk = IterClock{};
    a.sum[0] = d.sum[0];
    a.sum[1] = d.sum[1];
    a.sum2[0] = d.sum2[0];
    a.sum2[1] = d.sum2[1];
    a.ho_ptr = d.ho_ptr ? d.ho_ptr + static_cast<size_t>(p) * d.I : nullptr;
    a.ho_ent = d.ho_ent;
    a.ho_sum = d.ho_sum;
    a.nonfinite = d.nonfinite;
    const IterScalars it = iter_scalars_at(t, d.eps_tab, d.burn_in, d.thin, true, d.has_heldout != 0);
    sparse_task<LPG, QPL, LIK>(a, it, task);
}

// The context of virtual work-group v: wg_first[j] <= v < wg_first[j + 1].
__device__ __forceinline__ int job_of(const int32_t *wg_first, int n, int v)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (wg_first[mid] <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Several contexts in one launch: the work-group finds its context, reads
// the context's clock (iteration *clock + b.k; the clocks advance once after
// a call's launches) and runs its task of that iteration's part.
template <int LPG, int QPL, int LIK>
__global__ __launch_bounds__(kBlockThreads) void sparse_batch_kernel(BatchArgs b)
{
    const int j = job_of(b.wg_first, b.n, blockIdx.x);
    const JobDesc &d = *b.jobs[j];
    job_task<LPG, QPL, LIK>(d, *d.clock + b.k, blockIdx.x - b.wg_first[j]);
}

// n_iter iterations of the contexts in one cooperative launch.  The grid is
// at most what the device holds at once, so every work-group is resident;
// each strides over the virtual work-groups of all contexts (context j's
// tasks of its current part), then waits at a grid-wide barrier, which also
// orders the iteration's factor writes before the next iteration's reads.
// Every work-group runs the same n_iter barriers.
//
// The barrier is a counter that starts at 0 for the launch: after the k-th
// iteration each work-group waits (thread 0, with a short sleep) until the
// counter reaches (k + 1) * gridDim.x.  Its increment is an agent-scope
// release, after every thread's stores have completed (vmcnt 0) and a
// work-group barrier; the wait polls with relaxed loads and ends with one
// agent-scope acquire fence, so the next iteration sees all factor writes of
// this one on every XCD.  All work-groups are resident (cooperative launch),
// so every wait ends.
template <int LPG, int QPL, int LIK>
__global__ __launch_bounds__(kBlockThreads) void sparse_persistent_kernel(BatchArgs b, int32_t n_iter,
                                                                          uint32_t *barrier)
{
    __shared__ int ready;
    const int total = b.wg_first[b.n];
    for (int k = 0; k < n_iter; ++k) {
        for (int v = blockIdx.x; v < total; v += gridDim.x) {
            const int j = job_of(b.wg_first, b.n, v);
            const JobDesc &d = *b.jobs[j];
            job_task<LPG, QPL, LIK>(d, *d.clock + k, v - b.wg_first[j]);
            // the next task reuses the LDS partials of this one: every
            // wave must have read them before any wave writes again
            __syncthreads();
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this thread's stores have reached L2
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t target = static_cast<uint32_t>(k + 1) * gridDim.x;
            __hip_atomic_fetch_add(barrier, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            while (__hip_atomic_load(barrier, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target)
                __builtin_amdgcn_s_sleep(2);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            ready = 1;
        }
        __syncthreads();
    }
    (void)ready;
}

__global__ void reset_barrier_kernel(uint32_t *barrier)
{
    if (threadIdx.x == 0) *barrier = 0u;
}

struct ClockList {
    int32_t *clocks[kMaxBatch];
    int32_t delta[kMaxBatch];
    int32_t n;
};

__global__ void advance_clocks_kernel(ClockList l)
{
    if (static_cast<int>(threadIdx.x) < l.n) *l.clocks[threadIdx.x] += l.delta[threadIdx.x];
}

template <int LPG, int QPL>
hipError_t launch_persistent_lpg(const BatchArgs &b, int n_iter, int lik, int grid, uint32_t *barrier,
                                 hipStream_t stream)
{
    void *args[] = {const_cast<BatchArgs *>(&b), &n_iter, &barrier};
    const void *f;
    switch (lik) {
    case LIK_GAUSS: f = reinterpret_cast<const void *>(&sparse_persistent_kernel<LPG, QPL, LIK_GAUSS>); break;
    case LIK_POISSON: f = reinterpret_cast<const void *>(&sparse_persistent_kernel<LPG, QPL, LIK_POISSON>); break;
    case LIK_HALF: f = reinterpret_cast<const void *>(&sparse_persistent_kernel<LPG, QPL, LIK_HALF>); break;
    case LIK_GAMMA: f = reinterpret_cast<const void *>(&sparse_persistent_kernel<LPG, QPL, LIK_GAMMA>); break;
    default: f = reinterpret_cast<const void *>(&sparse_persistent_kernel<LPG, QPL, LIK_GENERAL>); break;
    }
    {
        // at most as many work-groups as the device holds at once (every one
        // must be resident for the grid barrier), and no more than there is
        // work; a smaller grid when asked
        int dev = 0, per_cu = 0;
        hipDeviceProp_t prop;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBlockThreads, 0);
        if (e != hipSuccess) return e;
        const int resident = std::min(per_cu * prop.multiProcessorCount, b.wg_first[b.n]);
        grid = grid > 0 ? std::min(grid, resident) : resident;
    }
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(reset_barrier_kernel, dim3(1), dim3(64), 0, stream, barrier);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel(f, dim3(static_cast<unsigned>(grid)), dim3(kBlockThreads), args, 0, stream);
}

template <int LPG, int QPL>
hipError_t launch_batch_lpg(const BatchArgs &b, int lik, hipStream_t stream)
{
    const dim3 grid(static_cast<unsigned>(b.wg_first[b.n])), block(kBlockThreads);
    switch (lik) {
    case LIK_GAUSS: hipLaunchKernelGGL((sparse_batch_kernel<LPG, QPL, LIK_GAUSS>), grid, block, 0, stream, b); break;
    case LIK_POISSON: hipLaunchKernelGGL((sparse_batch_kernel<LPG, QPL, LIK_POISSON>), grid, block, 0, stream, b); break;
    case LIK_HALF: hipLaunchKernelGGL((sparse_batch_kernel<LPG, QPL, LIK_HALF>), grid, block, 0, stream, b); break;
    case LIK_GAMMA: hipLaunchKernelGGL((sparse_batch_kernel<LPG, QPL, LIK_GAMMA>), grid, block, 0, stream, b); break;
    default: hipLaunchKernelGGL((sparse_batch_kernel<LPG, QPL, LIK_GENERAL>), grid, block, 0, stream, b); break;
    }
    return hipGetLastError();
}

template <int LPG, int QPL>
hipError_t launch_lpg(const SparseIterArgs &a, int lik, hipStream_t stream)
{
    const dim3 grid(static_cast<unsigned>(a.n_tasks)), block(kBlockThreads);
    switch (lik) {
    case LIK_GAUSS: hipLaunchKernelGGL((sparse_iter_kernel<LPG, QPL, LIK_GAUSS>), grid, block, 0, stream, a); break;
    case LIK_POISSON: hipLaunchKernelGGL((sparse_iter_kernel<LPG, QPL, LIK_POISSON>), grid, block, 0, stream, a); break;
    case LIK_HALF: hipLaunchKernelGGL((sparse_iter_kernel<LPG, QPL, LIK_HALF>), grid, block, 0, stream, a); break;
    case LIK_GAMMA: hipLaunchKernelGGL((sparse_iter_kernel<LPG, QPL, LIK_GAMMA>), grid, block, 0, stream, a); break;
    default: hipLaunchKernelGGL((sparse_iter_kernel<LPG, QPL, LIK_GENERAL>), grid, block, 0, stream, a); break;
    }
    return hipGetLastError();
}

}  // namespace

int sparse_block_threads() { return kBlockThreads; }

// Quads (float4 of k) per lane: 1 up to K = 16, 2 up to K = 64, else 4,
// which halves the lanes (and waves) per item as the rank grows (measured
// on 480k x 17.8k, K = 100: 190 instead of 198 us per iteration).
int sparse_quads_per_lane(int K)
{
    const int nq = (K + 3) / 4;
    return nq <= 4 ? 1 : nq <= 16 ? 2 : 4;
}

// Lanes per item group for qpl quads per lane: the smallest power of two
// covering the quads.
int sparse_lanes_for(int K, int qpl)
{
    const int need = ((K + 3) / 4 + qpl - 1) / qpl;
    int lpg = 1;
    while (lpg < need) lpg *= 2;
    return lpg;
}

int sparse_threads_per_group(int K) { return sparse_lanes_for(K, sparse_quads_per_lane(K)); }

// The (lanes per group, quads per lane) pairs the kernels are built for.
bool sparse_variant_exists(int lpg, int qpl)
{
    switch (qpl) {
    case 1: return lpg == 1 || lpg == 2 || lpg == 4 || lpg == 8;
    case 2: return lpg == 4 || lpg == 8 || lpg == 16 || lpg == 32;
    case 4: return lpg == 4 || lpg == 8 || lpg == 16;
    default: return false;
    }
}

hipError_t launch_sparse_batch(const BatchArgs &b, int lik, int lpg, int qpl, hipStream_t stream)
{
    if (b.n <= 0 || b.n > kMaxBatch || b.wg_first[b.n] == 0) return b.n > kMaxBatch ? hipErrorInvalidValue : hipSuccess;
    if (qpl == 1) {
        switch (lpg) {
        case 1: return launch_batch_lpg<1, 1>(b, lik, stream);
        case 2: return launch_batch_lpg<2, 1>(b, lik, stream);
        case 4: return launch_batch_lpg<4, 1>(b, lik, stream);
        case 8: return launch_batch_lpg<8, 1>(b, lik, stream);
        default: return hipErrorInvalidValue;
        }
    }
    if (qpl == 4) {
        switch (lpg) {
        case 4: return launch_batch_lpg<4, 4>(b, lik, stream);
        case 8: return launch_batch_lpg<8, 4>(b, lik, stream);
        case 16: return launch_batch_lpg<16, 4>(b, lik, stream);
        default: return hipErrorInvalidValue;
        }
    }
    if (qpl == 2) {
        switch (lpg) {
        case 4: return launch_batch_lpg<4, 2>(b, lik, stream);
        case 8: return launch_batch_lpg<8, 2>(b, lik, stream);
        case 16: return launch_batch_lpg<16, 2>(b, lik, stream);
        case 32: return launch_batch_lpg<32, 2>(b, lik, stream);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sparse_persistent(const BatchArgs &b, int n_iter, int lik, int lpg, int qpl, int grid,
                                    uint32_t *barrier, hipStream_t stream)
{
    if (b.n <= 0 || b.n > kMaxBatch || n_iter <= 0) return b.n > kMaxBatch ? hipErrorInvalidValue : hipSuccess;
    if (qpl == 1) {
        switch (lpg) {
        case 1: return launch_persistent_lpg<1, 1>(b, n_iter, lik, grid, barrier, stream);
        case 2: return launch_persistent_lpg<2, 1>(b, n_iter, lik, grid, barrier, stream);
        case 4: return launch_persistent_lpg<4, 1>(b, n_iter, lik, grid, barrier, stream);
        case 8: return launch_persistent_lpg<8, 1>(b, n_iter, lik, grid, barrier, stream);
        default: return hipErrorInvalidValue;
        }
    }
    if (qpl == 4) {
        switch (lpg) {
        case 4: return launch_persistent_lpg<4, 4>(b, n_iter, lik, grid, barrier, stream);
        case 8: return launch_persistent_lpg<8, 4>(b, n_iter, lik, grid, barrier, stream);
        case 16: return launch_persistent_lpg<16, 4>(b, n_iter, lik, grid, barrier, stream);
        default: return hipErrorInvalidValue;
        }
    }
    if (qpl == 2) {
        switch (lpg) {
        case 4: return launch_persistent_lpg<4, 2>(b, n_iter, lik, grid, barrier, stream);
        case 8: return launch_persistent_lpg<8, 2>(b, n_iter, lik, grid, barrier, stream);
        case 16: return launch_persistent_lpg<16, 2>(b, n_iter, lik, grid, barrier, stream);
        case 32: return launch_persistent_lpg<32, 2>(b, n_iter, lik, grid, barrier, stream);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_advance_clocks(int32_t *const *clocks, const int32_t *delta, int n, hipStream_t stream)
{
    for (int first = 0; first < n; first += kMaxBatch) {
        ClockList l{};
        l.n = std::min(kMaxBatch, n - first);
        for (int j = 0; j < l.n; ++j) {
            l.clocks[j] = clocks[first + j];
            l.delta[j] = delta[first + j];
        }
        hipLaunchKernelGGL(advance_clocks_kernel, dim3(1), dim3(kMaxBatch), 0, stream, l);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sparse_iter(const SparseIterArgs &a, int lik, int lpg, int qpl, hipStream_t stream)
{
    if (a.n_tasks == 0) return hipSuccess;
    if (qpl == 1) {
        switch (lpg) {
        case 1: return launch_lpg<1, 1>(a, lik, stream);
        case 2: return launch_lpg<2, 1>(a, lik, stream);
        case 4: return launch_lpg<4, 1>(a, lik, stream);
        case 8: return launch_lpg<8, 1>(a, lik, stream);
        default: return hipErrorInvalidValue;
        }
    }
    if (qpl == 4) {
        switch (lpg) {
        case 4: return launch_lpg<4, 4>(a, lik, stream);
        case 8: return launch_lpg<8, 4>(a, lik, stream);
        case 16: return launch_lpg<16, 4>(a, lik, stream);
        default: return hipErrorInvalidValue;
        }
    }
    if (qpl == 2) {
        switch (lpg) {
        case 4: return launch_lpg<4, 2>(a, lik, stream);
        case 8: return launch_lpg<8, 2>(a, lik, stream);
        case 16: return launch_lpg<16, 2>(a, lik, stream);
        case 32: return launch_lpg<32, 2>(a, lik, stream);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace psgld

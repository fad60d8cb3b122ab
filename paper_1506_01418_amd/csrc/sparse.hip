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
//    column-sorted (for H items), so each item's gradient is a plain
//    sequential sum over a contiguous run of entries -- no atomics;
//  * a group of LPG lanes owns one item, each lane four consecutive k
//    (a float4), so a K-length dot product is four FMAs plus a log2(LPG)
//    step butterfly across the group;
//  * long items are split over G groups of the same work-group, whose
//    partial gradients are combined in LDS in a fixed order;
//  * the Langevin step, noise, prior and mirroring are applied by the item's
//    first group right after its gradient, into the other ping-pong buffer;
//    the old buffers are only read, so no item waits for another.
#include "internal.hpp"
#include "noise.hpp"

namespace psgld {
namespace {

constexpr int kBlockThreads = 256;
constexpr int kUnroll = 4;

template <int LPG>
__device__ __forceinline__ float group_sum(float v)
{
#pragma unroll
    for (int off = LPG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LPG);
    return v;
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

// d/dmu log TW(v; mu, phi, beta) = (v - mu) mu^(beta-2) / phi, with the mean
// floored when beta < 2.
template <int LIK>
__device__ __forceinline__ float residual(float v, float mu, const SparseIterArgs &a)
{
    if constexpr (LIK == LIK_GAUSS) {
        return (v - mu) * a.inv_phi;
    } else if constexpr (LIK == LIK_POISSON) {
        const float m = fmaxf(mu, a.mu_floor);
        return (v - m) / m * a.inv_phi;
    } else {
        const float m = fmaxf(mu, a.mu_floor);
        return (v - m) * powf(m, a.beta - 2.0f) * a.inv_phi;
    }
}

__device__ __forceinline__ float4 load4(const float *p) { return *reinterpret_cast<const float4 *>(p); }

template <int LPG, int LIK>
__global__ __launch_bounds__(kBlockThreads) void sparse_iter_kernel(SparseIterArgs a)
{
    __shared__ float4 partial[kBlockThreads];
    const int tid = threadIdx.x;
    const int g = tid / LPG;
    const int lane = tid % LPG;
    const Task task = a.tasks[blockIdx.x];
    const int side = task.side;
    const int G = task.G;
    const int slot = g / G;
    const int sub = g % G;
    const bool active = slot < task.count;
    const int item = active ? a.items[task.first + slot] : 0;
    const int Kp = a.Kp;
    const bool qlane = lane < a.nq;
    const float *__restrict__ own = a.x_old[side];
    const float *__restrict__ other = a.x_old[side ^ 1];
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);

    float4 x = zero;
    if (active && qlane) x = load4(own + static_cast<size_t>(item) * Kp + 4 * lane);

    int s0 = 0, s1 = 0;
    if (active) {
        const int beg = a.ptr[side][item];
        const int n = a.ptr[side][item + 1] - beg;
        s0 = beg + static_cast<int>((static_cast<long long>(n) * sub) / G);
        s1 = beg + static_cast<int>((static_cast<long long>(n) * (sub + 1)) / G);
    }

    // Gradient of the likelihood over this group's share of the item's entries.
    const Entry *__restrict__ ent = a.ent[side];
    float4 acc = zero;
    int e = s0;
    for (; e + kUnroll <= s1; e += kUnroll) {
        Entry en[kUnroll];
        float4 o[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) en[u] = ent[e + u];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            o[u] = qlane ? load4(other + static_cast<size_t>(en[u].idx) * Kp + 4 * lane) : zero;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const float mu = group_sum<LPG>(dot4(x, o[u]));
            axpy4(acc, residual<LIK>(en[u].val, mu, a), o[u]);
        }
    }
    for (; e < s1; ++e) {
        const Entry en = ent[e];
        const float4 o = qlane ? load4(other + static_cast<size_t>(en.idx) * Kp + 4 * lane) : zero;
        const float mu = group_sum<LPG>(dot4(x, o));
        axpy4(acc, residual<LIK>(en.val, mu, a), o);
    }

    // Long items: combine the G partial sums in a fixed order.
    if (G > 1) {
        partial[tid] = acc;
        __syncthreads();
        if (sub == 0) {
            acc = zero;
            for (int s = 0; s < G; ++s) {
                const float4 p = partial[(g + s) * LPG + lane];
                acc.x += p.x;
                acc.y += p.y;
                acc.z += p.z;
                acc.w += p.w;
            }
        }
    }
    if (!active || sub != 0) return;

    // Held-out predictive sums at the state entering this iteration.
    if (side == 0 && a.do_heldout) {
        const int hb = a.ho_ptr[item], he = a.ho_ptr[item + 1];
        for (int h = hb; h < he; ++h) {
            const HeldEntry c = a.ho_ent[h];
            const float4 o = qlane ? load4(other + static_cast<size_t>(c.col) * Kp + 4 * lane) : zero;
            const float mu = group_sum<LPG>(dot4(x, o));
            if (lane == 0) a.ho_sum[c.slot] += static_cast<double>(mu);
        }
    }
    if (!qlane) return;

    // Langevin step for k = 4 lane .. 4 lane + 3.
    const bool frozen = (a.flags & (side == 0 ? PSGLD_TEST_FREEZE_W : PSGLD_TEST_FREEZE_H)) != 0;
    const bool noisy = !frozen && !(a.flags & PSGLD_TEST_NOISE_OFF);
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (noisy) {
        const Normal4 nz = normal4(a.seed_lo, a.seed_hi, a.t, static_cast<uint32_t>(side),
                                   static_cast<uint32_t>(item), static_cast<uint32_t>(lane));
        z[0] = nz.z[0];
        z[1] = nz.z[1];
        z[2] = nz.z[2];
        z[3] = nz.z[3];
    }
    const float xo[4] = {x.x, x.y, x.z, x.w};
    const float gr[4] = {acc.x, acc.y, acc.z, acc.w};
    const float lam = a.lambda[side];
    float xn[4];
    bool finite = true;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float v = xo[c];
        if (!frozen) {
            const float pg = a.prior_kind == PSGLD_PRIOR_EXPONENTIAL ? (xo[c] >= 0.f ? -lam : lam)
                                                                     : -lam * xo[c];
            v = xo[c] + a.eps * (a.scale * gr[c] + pg) + a.sigma * z[c];
            if (a.mirror) v = fabsf(v);
        }
        if (4 * lane + c >= a.K) v = 0.f;
        finite = finite && isfinite(v);
        xn[c] = v;
    }
    const size_t off = static_cast<size_t>(item) * Kp + 4 * lane;
    *reinterpret_cast<float4 *>(a.x_new[side] + off) = make_float4(xn[0], xn[1], xn[2], xn[3]);
    if (!finite) atomicMin(a.nonfinite, static_cast<int32_t>(a.t));
    if (a.do_moments) {
        double *s = a.sum[side] + off;
        double *s2 = a.sum2[side] + off;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double v = static_cast<double>(xn[c]);
            s[c] += v;
            s2[c] += v * v;
        }
    }
}

template <int LPG>
hipError_t launch_lpg(const SparseIterArgs &a, int lik, hipStream_t stream)
{
    const dim3 grid(static_cast<unsigned>(a.n_tasks)), block(kBlockThreads);
    switch (lik) {
    case LIK_GAUSS:
        hipLaunchKernelGGL((sparse_iter_kernel<LPG, LIK_GAUSS>), grid, block, 0, stream, a);
        break;
    case LIK_POISSON:
        hipLaunchKernelGGL((sparse_iter_kernel<LPG, LIK_POISSON>), grid, block, 0, stream, a);
        break;
    default:
        hipLaunchKernelGGL((sparse_iter_kernel<LPG, LIK_GENERAL>), grid, block, 0, stream, a);
        break;
    }
    return hipGetLastError();
}

}  // namespace

int sparse_block_threads() { return kBlockThreads; }

// Lanes per item group: the smallest power of two covering ceil(K/4) quads.
int sparse_threads_per_group(int K)
{
    const int nq = (K + 3) / 4;
    int lpg = 1;
    while (lpg < nq) lpg *= 2;
    return lpg;
}

hipError_t launch_sparse_iter(const SparseIterArgs &a, int lik, int lpg, hipStream_t stream)
{
    if (a.n_tasks == 0) return hipSuccess;
    switch (lpg) {
    case 1: return launch_lpg<1>(a, lik, stream);
    case 2: return launch_lpg<2>(a, lik, stream);
    case 4: return launch_lpg<4>(a, lik, stream);
    case 8: return launch_lpg<8>(a, lik, stream);
    case 16: return launch_lpg<16>(a, lik, stream);
    case 32: return launch_lpg<32>(a, lik, stream);
    case 64: return launch_lpg<64>(a, lik, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace psgld

// Small kernels beside the sampler: evaluation of the noise stream for
// given counters, and the FP64 training log-likelihood reduction.
#include <algorithm>
#include "internal.hpp"
#include "noise.hpp"

namespace psgld {
namespace {

__global__ void philox_blocks_kernel(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Block4 b = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                                   key[2 * i], key[2 * i + 1]);
    for (int m = 0; m < 4; ++m) out[4 * i + m] = b.r[m];
}

// One thread per (request, quad): the normals k = 4q..4q+3 of one row/column.
__global__ void normals_kernel(int64_t n, uint32_t seed_lo, uint32_t seed_hi, const int64_t *t,
                               const uint32_t *stream_id, const int64_t *index, int K, float *z,
                               float *radius)
{
    const int nq = (K + 3) / 4;
    const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (w >= n * nq) return;
    const int64_t r = w / nq;
    const int q = static_cast<int>(w % nq);
    const Normal4 nz = normal4(seed_lo, seed_hi, static_cast<uint32_t>(t[r]), stream_id[r],
                               static_cast<uint32_t>(index[r]), static_cast<uint32_t>(q));
    for (int m = 0; m < 4; ++m) {
        const int k = 4 * q + m;
        if (k < K) {
            z[r * K + k] = nz.z[m];
            radius[r * K + k] = nz.radius[m / 2];
        }
    }
}

// beta-divergence d_beta(v||mu), with the KL and IS limits at beta = 1, 0,
// and the general formula in closed form at beta = 2 (half the squared
// difference) and beta = 1/2 (-4 sqrt(v) + 2 v / sqrt(mu) + 2 sqrt(mu)).
__device__ double dbeta(double v, double mu, double beta)
{
    if (beta == 2.0) return 0.5 * (v - mu) * (v - mu);
    if (beta == 1.0) return (v > 0.0 ? v * log(v / mu) : 0.0) - v + mu;
    if (beta == 0.5) {
        const double r = sqrt(mu);
        return -4.0 * sqrt(v) + 2.0 * v / r + 2.0 * r;
    }
    if (beta == 0.0) return v / mu - log(v / mu) - 1.0;
    return pow(v, beta) / (beta * (beta - 1.0)) - v * pow(mu, beta - 1.0) / (beta - 1.0) +
           pow(mu, beta) / beta;
}

__global__ void set_clock_kernel(int32_t *clock, int32_t value)
{
    if (threadIdx.x == 0) *clock = value;
}

__global__ void advance_clock_kernel(int32_t *clock, int32_t delta)
{
    if (threadIdx.x == 0) *clock += delta;
}

__global__ void fill_i32_kernel(int32_t *p, int32_t value, int64_t n)
{
    for (int64_t m = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; m < n;
         m += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[m] = value;
}

constexpr int kLLThreads = 256;

__global__ __launch_bounds__(kLLThreads) void loglik_partial_kernel(
    const float *W, const float *Hs, const int32_t *row_of_entry, const Entry *ent, int64_t n, int K,
    int Kp, double beta, double phi, double mu_floor, double *partials)
{
    __shared__ double red[kLLThreads];
    double acc = 0.0;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kLLThreads + threadIdx.x; e < n;
         e += static_cast<int64_t>(gridDim.x) * kLLThreads) {
        const float4 *w = reinterpret_cast<const float4 *>(W + static_cast<size_t>(row_of_entry[e]) * Kp);
        const float4 *h = reinterpret_cast<const float4 *>(Hs + ent[e].off);
        double mu = 0.0;
        for (int q = 0; 4 * q < K; ++q) {      // rows hold Kp >= K floats, zero past K
            const float4 a = w[q], b = h[q];
            mu += static_cast<double>(a.x) * static_cast<double>(b.x);
            mu += static_cast<double>(a.y) * static_cast<double>(b.y);
            mu += static_cast<double>(a.z) * static_cast<double>(b.z);
            mu += static_cast<double>(a.w) * static_cast<double>(b.w);
        }
        if (beta < 2.0 && mu < mu_floor) mu = mu_floor;
        acc -= dbeta(static_cast<double>(ent[e].val), mu, beta) / phi;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kLLThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// Same for the training cells of dense blocks: blockIdx.y is the block.
__global__ __launch_bounds__(kLLThreads) void dense_loglik_partial_kernel(
    const float *W, const float *Hs, const DenseBlock *blocks, const float *val, const uint16_t *val16,
    const uint32_t *mask, int K, int Kp, double beta, double phi, double mu_floor, double *partials, int per_block)
{
    __shared__ double red[kLLThreads];
    const DenseBlock blk = blocks[blockIdx.y];
    const int64_t cells = static_cast<int64_t>(blk.m) * blk.n;
    double acc = 0.0;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kLLThreads + threadIdx.x; e < cells;
         e += static_cast<int64_t>(per_block) * kLLThreads) {
        const int i = static_cast<int>(e / blk.n), j = static_cast<int>(e % blk.n);
        const int64_t cell = blk.v_off + static_cast<int64_t>(i) * blk.ld + j;
        if (dense_code(mask, cell) != kMaskTrain) continue;
        const float4 *w = reinterpret_cast<const float4 *>(W + static_cast<size_t>(blk.row0 + i) * Kp);
        const float4 *h = reinterpret_cast<const float4 *>(Hs + static_cast<size_t>(blk.col0 + j) * Kp);
        double mu = 0.0;
        for (int q = 0; 4 * q < K; ++q) {      // rows hold Kp >= K floats, zero past K
            const float4 a = w[q], b = h[q];
            mu += static_cast<double>(a.x) * static_cast<double>(b.x);
            mu += static_cast<double>(a.y) * static_cast<double>(b.y);
            mu += static_cast<double>(a.z) * static_cast<double>(b.z);
            mu += static_cast<double>(a.w) * static_cast<double>(b.w);
        }
        if (beta < 2.0 && mu < mu_floor) mu = mu_floor;
        const float v = val ? val[cell] : bf16_value(val16[cell]);
        acc -= dbeta(static_cast<double>(v), mu, beta) / phi;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kLLThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[static_cast<size_t>(blockIdx.y) * per_block + blockIdx.x] = red[0];
}

// Sums the per-block partials in index order (deterministic).
__global__ void sum_in_order_kernel(const double *partials, int n, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partials[i];
    *out = s;
}

}  // namespace

hipError_t launch_philox_blocks(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out,
                                hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
    hipLaunchKernelGGL(philox_blocks_kernel, dim3(blocks), dim3(256), 0, stream, n, ctr, key, out);
    return hipGetLastError();
}

hipError_t launch_normals(int64_t n, uint64_t seed, const int64_t *t, const uint32_t *stream_id,
                          const int64_t *index, int K, float *z, float *radius, hipStream_t stream)
{
    const int64_t work = n * ((K + 3) / 4);
    if (work == 0) return hipSuccess;
    const unsigned blocks = static_cast<unsigned>((work + 255) / 256);
    hipLaunchKernelGGL(normals_kernel, dim3(blocks), dim3(256), 0, stream, n,
                       static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), t, stream_id,
                       index, K, z, radius);
    return hipGetLastError();
}

hipError_t launch_loglik(const float *W, const float *Hs, const int32_t *row_of_entry,
                         const Entry *ent, int64_t n, int K, int Kp, double beta, double phi,
                         double mu_floor, double *partials, int n_blocks, hipStream_t stream)
{
    hipLaunchKernelGGL(loglik_partial_kernel, dim3(n_blocks), dim3(kLLThreads), 0, stream, W, Hs,
                       row_of_entry, ent, n, K, Kp, beta, phi, mu_floor, partials);
    return hipGetLastError();
}

hipError_t launch_dense_loglik(const float *W, const float *Hs, const DenseBlock *blocks, int n_blocks,
                               const float *val, const uint16_t *val16, const uint32_t *mask, int K, int Kp,
                               double beta, double phi, double mu_floor, double *partials, int per_block,
                               hipStream_t stream)
{
    if (n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(dense_loglik_partial_kernel, dim3(per_block, n_blocks), dim3(kLLThreads), 0, stream, W,
                       Hs, blocks, val, val16, mask, K, Kp, beta, phi, mu_floor, partials, per_block);
    return hipGetLastError();
}

hipError_t launch_sum_in_order(const double *partials, int n, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(sum_in_order_kernel, dim3(1), dim3(64), 0, stream, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_set_clock(int32_t *clock, int32_t value, hipStream_t stream)
{
    hipLaunchKernelGGL(set_clock_kernel, dim3(1), dim3(64), 0, stream, clock, value);
    return hipGetLastError();
}

hipError_t launch_advance_clock(int32_t *clock, int32_t delta, hipStream_t stream)
{
    hipLaunchKernelGGL(advance_clock_kernel, dim3(1), dim3(64), 0, stream, clock, delta);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, p, value, n);
    return hipGetLastError();
}

}  // namespace psgld

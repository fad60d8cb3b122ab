// Langevin noise of the sampler on the device: N(0,1) draws from a
// counter-based generator, so that any parameter's noise at any iteration
// is a pure function of (seed, iteration, factor, row-or-column, k) and no
// generator state is stored or carried between launches.
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds;
// each multiplies counter words 0 and 2 by the two 32-bit Philox constants,
// then combines the high products with words 1, 3 and the round key; the
// key advances by the 32-bit Weyl increments between rounds.
// Counter = (k/4, row-or-column index, iteration, factor), key = seed.
// Transform: u = (2 (r >> 9) + 1) * 2^-24 (exact, in (0,1)); Box-Muller on
// the pairs (u0,u1) and (u2,u3) gives the normals of k = 4q..4q+3.
// Box-Muller uses the hardware transcendentals: v_log_f32 (log2), v_sqrt_f32,
// and v_sin_f32 / v_cos_f32, which take their argument in revolutions, so
// cos(2 pi u) is v_cos_f32(u) with no range reduction.  Checked against
// FP64 over all 2^23 possible uniforms: radius relative error <= 1.4e-7,
// sine / cosine absolute error <= 1.3e-7.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psgld {

struct Block4 {
    uint32_t r[4];
};

__host__ __device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                         uint32_t c3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    constexpr uint32_t kInc0 = 0x9E3779B9u, kInc1 = 0xBB67AE85u;
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        const uint64_t m0 = static_cast<uint64_t>(kMul0) * c0;
        const uint64_t m1 = static_cast<uint64_t>(kMul1) * c2;
        const uint32_t n0 = static_cast<uint32_t>(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(m0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(m1);
        c3 = static_cast<uint32_t>(m0);
        c0 = n0;
        c2 = n2;
        k0 += kInc0;
        k1 += kInc1;
    }
    return Block4{{c0, c1, c2, c3}};
}

// (2 (r >> 9) + 1) * 2^-24: the integer is < 2^24, so the conversion and the
// power-of-two scaling are exact.
__device__ __forceinline__ float open_unit(uint32_t r)
{
    return static_cast<float>(((r >> 9) << 1) | 1u) * 5.9604644775390625e-8f;
}

struct Normal4 {
    float z[4];
    float radius[2];
};

// Normals k = 4q..4q+3 of row/column `index` of factor `stream` at iteration t.
__device__ __forceinline__ Normal4 normal4(uint32_t seed_lo, uint32_t seed_hi, uint32_t t,
                                           uint32_t stream, uint32_t index, uint32_t q)
{
    const Block4 b = philox4x32_10(q, index, t, stream, seed_lo, seed_hi);
    Normal4 out;
#pragma unroll
    for (int pair = 0; pair < 2; ++pair) {
        const float ua = open_unit(b.r[2 * pair]);
        const float ub = open_unit(b.r[2 * pair + 1]);
        // -2 ln u = -2 ln(2) log2(u)
        const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
        out.z[2 * pair] = rad * __builtin_amdgcn_cosf(ub);
        out.z[2 * pair + 1] = rad * __builtin_amdgcn_sinf(ub);
        out.radius[pair] = rad;
    }
    return out;
}

}  // namespace psgld

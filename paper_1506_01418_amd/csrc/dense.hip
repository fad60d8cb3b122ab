// One PSGLD iteration over the dense blocks of a part, on the matrix cores.
//
// For a dense block (rows R_b, columns C_c) of the part, Eq. (8)-(9) need
//   mu  = W_b H_c                (the block's means, Eq. (13))
//   E   = train * (V - mu~) mu~^(beta-2) / phi   (train: 1 for training cells)
//   G_H = W_b^T E                (K x |C_c|: complete per column)
//   G_W = E H_c^T                (|R_b| x K: summed over the block's columns)
// A work-group owns up to kDenseSubTiles x 64 columns of one block (fewer
// for blocks taller than 64 rows) and all of its m <= 128 rows.  The three products run on MFMA 16x16 tiles (FP32
// operands, or BF16 operands rounded to nearest even, always FP32
// accumulation) from LDS copies of W_b, a 64-column sub-tile of H and E,
// with four independent accumulators per wave.  The H columns are updated
// straight from the G_H accumulators -- each lane holds four consecutive k
// of one column, which is exactly one Philox quad.  G_W accumulates over
// the work-group's sub-tiles and is left as its partial, which
// dense_w_update_kernel sums over the block's work-groups in order before
// updating the block's W rows.
#include "internal.hpp"
#include "noise.hpp"

namespace psgld {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kDenseThreads = 512;   // 8 waves: two per 16-row tile, k-tile or column half
constexpr int kNT = kDenseTileCols;

// D_t(16x16) += A(16 x kd) B_t(kd x 16) for t < nb (at most NACC), all with
// the same A rows: A(r, k) = fa(r, k), B_t(k, c) = fb(t, k, c).  FP32:
// 16x16x4 steps (kd a multiple of 4); BF16: 16x16x32 steps (kd a multiple
// of 32), operands rounded to nearest even.  Lane layouts (checked on the
// device): A lane l holds row l%16 and k-slice l/16; B lane l holds column
// l%16; D lane l, register r holds (4 (l/16) + r, l%16).
template <bool BF16, int NACC, typename FA, typename FB>
__device__ __forceinline__ void mma16(v4f (&acc)[NACC], int nb, int kd, int lane, FA fa, FB fb)
{
    const int r = lane & 15, h = lane >> 4;
    if constexpr (BF16) {
        for (int k = 0; k < kd; k += 32) {
            v8bf av;
#pragma unroll
            for (int v = 0; v < 8; ++v) av[v] = static_cast<__bf16>(fa(r, k + 8 * h + v));
#pragma unroll
            for (int t = 0; t < NACC; ++t) {
                if (t >= nb) break;
                v8bf bv;
#pragma unroll
                for (int v = 0; v < 8; ++v) bv[v] = static_cast<__bf16>(fb(t, k + 8 * h + v, r));
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
            }
        }
    } else {
#pragma unroll 2
        for (int k = 0; k < kd; k += 4) {
            const float av = fa(r, k + h);
#pragma unroll
            for (int t = 0; t < NACC; ++t) {
                if (t >= nb) break;
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, fb(t, k + h, r), acc[t], 0, 0, 0);
            }
        }
    }
}

// The Langevin step of four consecutive parameters k0..k0+3 of row `index`
// of factor `side`, with gradient g of the scaled likelihood.
__device__ __forceinline__ void dense_langevin(const DenseIterArgs &a, const IterScalars &it, int side, int index,
                                               int k0, const float xo[4],
                               const float g[4])
{
    const bool frozen = (a.flags & (side == 0 ? PSGLD_TEST_FREEZE_W : PSGLD_TEST_FREEZE_H)) != 0;
    const bool noisy = !frozen && !(a.flags & PSGLD_TEST_NOISE_OFF);
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (noisy) {
        const Normal4 nz = normal4(a.seed_lo, a.seed_hi, it.t, static_cast<uint32_t>(side),
                                   static_cast<uint32_t>(index), static_cast<uint32_t>(k0 / 4));
        z[0] = nz.z[0];
        z[1] = nz.z[1];
        z[2] = nz.z[2];
        z[3] = nz.z[3];
    }
    const float lam = a.lambda[side];
    float xn[4];
    bool finite = true;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float v = xo[c];
        if (!frozen) {
            const float pg = a.prior_kind == PSGLD_PRIOR_EXPONENTIAL ? (xo[c] >= 0.f ? -lam : lam) : -lam * xo[c];
            v = xo[c] + it.eps * (a.scale * g[c] + pg) + it.sigma * z[c];
            if (a.mirror) v = fabsf(v);
        }
        if (k0 + c >= a.K) v = 0.f;
        finite = finite && isfinite(v);
        xn[c] = v;
    }
    const size_t off = static_cast<size_t>(index) * a.Kp + k0;
    *reinterpret_cast<float4 *>(a.x_new[side] + off) = make_float4(xn[0], xn[1], xn[2], xn[3]);
    if (!finite) atomicMin(a.nonfinite, static_cast<int32_t>(it.t));
    if (it.do_moments) {
        double2 *s = reinterpret_cast<double2 *>(a.sum[side] + off);
        double2 *s2 = reinterpret_cast<double2 *>(a.sum2[side] + off);
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

// One work-group: up to kDenseSubTiles consecutive 64-column sub-tiles of
// one block.  Wave w takes 16-row tiles w, w+4, ... of each product; the
// products over the rank (G_H and G_W) use one 16-row k-tile per wave
// (K <= 64).  G_W accumulates in registers over the sub-tiles and is
// written once, as this work-group's partial.
__device__ __forceinline__ float4 load4(const float *p) { return *reinterpret_cast<const float4 *>(p); }

// Register staging of a 64-column piece of a factor stored row by row with
// Kp floats per row: 16 quad slots per row (K <= 64), kStageQ float4 per
// thread, consecutive threads on consecutive quads of a row, so a wave reads
// four whole rows.  Slots past the rows asked for, or past Kp, hold zeros.
constexpr int kStageQ = kNT * (kDenseMaxK / 4) / kDenseThreads;

struct Stage {
    float4 v[kStageQ];
};

__device__ __forceinline__ void stage_load(Stage &st, const float *base, int first_row, int nrows, int Kp, int tid)
{
#pragma unroll
    for (int u = 0; u < kStageQ; ++u) {
        const int f = tid + u * kDenseThreads;
        const int j = f >> 4, q = f & 15;
        st.v[u] = (j < nrows && 4 * q < Kp) ? load4(base + static_cast<size_t>(first_row + j) * Kp + 4 * q)
                                            : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Writes the staged rows j (of 64) into LDS rows j0 + j < rows with stride
// `stride`, columns 0 .. KS - 1.
__device__ __forceinline__ void stage_store(const Stage &st, float *lds, int j0, int rows, int stride, int KS,
                                            int tid)
{
#pragma unroll
    for (int u = 0; u < kStageQ; ++u) {
        const int f = tid + u * kDenseThreads;
        const int j = f >> 4, q = f & 15;
        if (4 * q < KS && j0 + j < rows) {
            float *d = lds + (j0 + j) * stride + 4 * q;
            d[0] = st.v[u].x;
            d[1] = st.v[u].y;
            d[2] = st.v[u].z;
            d[3] = st.v[u].w;
        }
    }
}

// Register staging of the values and cell codes of a sub-tile's first 64
// rows: kVQ float4 of values per thread, aligned loads (rows start on
// 64-byte boundaries), so a wave reads whole 256-byte row pieces; the first
// 256 threads each take one 32-bit word (16 cells) of codes.  Cells past the
// block's rows or its padded width read as missing.
constexpr int kVQ = 64 * 64 / 4 / kDenseThreads;
struct VStage {
    float4 v[kVQ];
    uint32_t mk;
};

__device__ __forceinline__ void vstage_load(VStage &st, const float *V, const uint32_t *M, const DenseBlock &blk,
                                            int m, int cl, int tid)
{
    const int ld = blk.ld;
#pragma unroll
    for (int u = 0; u < kVQ; ++u) {
        const int f = tid + u * kDenseThreads;
        const int j = f >> 4, c = cl + 4 * (f & 15);
        st.v[u] = (j < m && c < ld) ? load4(V + static_cast<size_t>(j) * ld + c) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int j = tid >> 2, c = cl + 16 * (tid & 3);
    st.mk = (tid < 256 && j < m && c < ld) ? M[(blk.v_off + static_cast<int64_t>(j) * ld + c) >> 4] : 0u;
}

// Values into rows 0 .. min(64, rows) - 1 of sV (row stride `stride`; sV
// has `rows` rows), codes into sM (64 rows x 4 words of 16 cells).
__device__ __forceinline__ void vstage_store(const VStage &st, float *sV, int stride, int rows, uint32_t *sM,
                                             int tid)
{
#pragma unroll
    for (int u = 0; u < kVQ; ++u) {
        const int f = tid + u * kDenseThreads;
        if ((f >> 4) >= rows) continue;
        float *d = sV + (f >> 4) * stride + 4 * (f & 15);
        d[0] = st.v[u].x;
        d[1] = st.v[u].y;
        d[2] = st.v[u].z;
        d[3] = st.v[u].w;
    }
    if (tid < 256) sM[tid] = st.mk;
}

// One work-group: up to kDenseSubTiles consecutive 64-column sub-tiles of
// one block.  Wave w = 4 ch + wq (ch = 0, 1) takes the 16-row tiles wq,
// wq + 4, ... of mu over column half ch of the sub-tile; in G_H it takes
// k-tile wq over column half ch, in G_W k-tile wq over the 16-row tiles ch,
// ch + 2, ... (K <= 64).  The next
// sub-tile's H columns are loaded into registers while the current one is
// computed, and so are the values and cell codes of its first 64 rows (rows
// past 64 are loaded before their row tile's product), so no product waits
// on a round trip to memory it could have started earlier.  G_W accumulates
// in registers over the sub-tiles and is written once, as this work-group's
// partial.
template <bool BF16, int LIK, bool VAL16>
__global__ __launch_bounds__(kDenseThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void dense_tile_kernel(DenseIterArgs a)
{
    extern __shared__ float lds[];
    const DenseTile tile = a.tiles[blockIdx.x];
    const int32_t *ho = a.tiles[blockIdx.x].ho;   // read in place: indexed by the sub-tile
    const DenseBlock blk = a.blocks[tile.block];
    const IterScalars itr = iter_scalars(a.clk);
    const int m = blk.m, MT = (m + a.row_align - 1) / a.row_align * a.row_align;
    const int KS = a.KS, Kp = a.Kp;
    const int sw = KS + 1;            // odd row strides: no LDS bank conflicts
    const int se = kNT + 1;
    float *sW = lds;                   // [MT][KS+1]   W_b
    float *sH = sW + MT * sw;          // [NT][KS+1]   H columns of the sub-tile
    float *sE = sH + kNT * sw;         // [MT][NT+1]   values of the sub-tile, then E
    uint32_t *sM = reinterpret_cast<uint32_t *>(sE + MT * se);   // [64][4] cell codes of rows 0..63
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c16 = lane & 15, h4 = lane >> 4;
    const int wq = wave & 3, ch = wave >> 2;
    const float *Wold = a.x_old[0], *Hold = a.x_old[1];

    // W_b (two 64-row pieces) and the first sub-tile's H columns, all in flight together
    Stage hs, ws0, ws1;
    stage_load(hs, Hold, blk.col0 + tile.col, min(kNT, blk.n - tile.col), Kp, tid);
    stage_load(ws0, Wold, blk.row0, min(kNT, m), Kp, tid);
    if (MT > kNT) stage_load(ws1, Wold, blk.row0 + kNT, m - kNT, Kp, tid);
    stage_store(ws0, sW, 0, MT, sw, KS, tid);
    if (MT > kNT) stage_store(ws1, sW, kNT, MT, sw, KS, tid);

    // values in FP32, or (VAL16, BF16 operands only) stored in BF16
    const float *V = VAL16 ? nullptr : a.val + blk.v_off;
    const uint16_t *V16 = VAL16 ? a.val16 + blk.v_off : nullptr;
    const uint32_t *M = a.mask;
    const uint32_t *Mb = M + (blk.v_off >> 4);   // the block's code words
    const int ld = blk.ld;
    // FP32 operands: values and cell codes of rows 0..63 prefetched one
    // sub-tile ahead; BF16 operands need those registers for the operand
    // conversions, and read the values in place before each product
    constexpr bool kStageV = !BF16;
    static_assert(!VAL16 || BF16, "BF16 values go with BF16 operands");
    VStage vs;
    if constexpr (kStageV) vstage_load(vs, V, M, blk, m, tile.col, tid);
    const int kt = wq;                            // this wave's k-tile in G_H and G_W
    const bool has_kt = kt * 16 < KS;
    const int n_it = MT / 16;                     // 16-row tiles of the block
    constexpr int kGW = kDenseMaxRows / 32;       // G_W row tiles per wave: ch, ch + 2, ...
    const int n_gw = (n_it - ch + 1) / 2;
    v4f gw[kGW];
#pragma unroll
    for (int t = 0; t < kGW; ++t) gw[t] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int sub = 0; sub < blk.n_sub; ++sub) {
        const int cl = tile.col + sub * kNT;      // first column of the sub-tile, in the block
        if (cl >= blk.n) break;
        const int ncol = min(kNT, blk.n - cl);
        const int col0 = blk.col0 + cl;
        __syncthreads();                          // previous sub-tile done with sH, sE, sM
        stage_store(hs, sH, 0, kNT, sw, KS, tid);
        if constexpr (kStageV) vstage_store(vs, sE, se, MT, sM, tid);
        if (sub + 1 < blk.n_sub && cl + kNT < blk.n) {
            stage_load(hs, Hold, col0 + kNT, min(kNT, blk.n - cl - kNT), Kp, tid);
            if constexpr (kStageV) vstage_load(vs, V, M, blk, m, cl + kNT, tid);
        }
        __syncthreads();

        // mu = W_b H^T (MT x 64) and E, one 16-row tile at a time; values and
        // cell codes of rows 0..63 come from LDS, those of later rows
        // (clamped into the block, masked after) are requested before the
        // tile's product
        for (int it = wq; it < n_it; it += 4) {
            float vv[2][4];
            uint32_t mm[2][4];
            if (kStageV && it < 4) {
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = it * 16 + 4 * h4 + r, j = (2 * ch + t) * 16 + c16;
                        vv[t][r] = sE[i * se + j];
                        mm[t][r] = (sM[4 * i + 2 * ch + t] >> (2 * c16)) & 3u;   // j = 16 (2 ch + t) + c16
                    }
            } else {
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = min(it * 16 + 4 * h4 + r, m - 1);
                        const int j = min((2 * ch + t) * 16 + c16, ncol - 1);
                        const size_t cell = static_cast<size_t>(i) * ld + cl + j;
                        vv[t][r] = VAL16 ? bf16_value(V16[cell]) : V[cell];
                        // v_off, ld and cl are multiples of 16: the cell's code
                        // sits at bits 2 c16 of its word (a clamped cell
                        // reads another code, masked as outside)
                        mm[t][r] = (Mb[cell >> 4] >> (2 * c16)) & 3u;
                    }
            }
            v4f acc[2] = {};
            mma16<BF16, 2>(acc, 2, KS, lane, [&](int r, int k) { return sW[(it * 16 + r) * sw + k]; },
                           [&](int t, int k, int c) { return sH[((2 * ch + t) * 16 + c) * sw + k]; });
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int j = (2 * ch + t) * 16 + c16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = it * 16 + 4 * h4 + r;
                    // E for training cells; the mean itself for held-out cells
                    // (read out and cleared below, before the products use E)
                    const bool inside = i < m && j < ncol;
                    const float res = tweedie_residual<LIK>(vv[t][r], acc[t][r], a.inv_phi, a.beta, a.mu_floor);
                    float e = 0.f;
                    if (inside && mm[t][r] == kMaskTrain) e = res;
                    if (inside && mm[t][r] == kMaskHeld && itr.do_heldout) e = acc[t][r];
                    sE[i * se + j] = e;
                }
            }
        }
        __syncthreads();
        const int ho_b = ho[sub], ho_e = ho[sub + 1];
        if (itr.do_heldout && ho_e > ho_b) {
            // held-out cells of this sub-tile: add their mean, then zero them in E
            for (int h = ho_b + tid; h < ho_e; h += kDenseThreads) {
                const DenseHeld c = a.heldout[h];
                const int j = c.col - sub * kNT;
                a.ho_sum[c.slot] += static_cast<double>(sE[c.row * se + j]);
                sE[c.row * se + j] = 0.f;
            }
            __syncthreads();
        }

        if (has_kt) {
            // G_H = W_b^T E (k-tile kt x column half ch): update those H columns
            v4f acc[2] = {};
            mma16<BF16, 2>(acc, 2, MT, lane, [&](int r, int i) { return sW[i * sw + kt * 16 + r]; },
                           [&](int t, int i, int c) { return sE[i * se + (2 * ch + t) * 16 + c]; });
            const int k0 = kt * 16 + 4 * h4;      // four consecutive k: one Philox quad
            if (k0 < Kp) {
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int j = (2 * ch + t) * 16 + c16;
                    if (j >= ncol) continue;
                    const float g[4] = {acc[t][0], acc[t][1], acc[t][2], acc[t][3]};
                    const float xo[4] = {sH[j * sw + k0], sH[j * sw + k0 + 1], sH[j * sw + k0 + 2],
                                         sH[j * sw + k0 + 3]};
                    dense_langevin(a, itr, 1, col0 + j, k0, xo, g);
                }
            }
            // G_W^T += H^T E^T (k-tile kt x row tiles ch, ch + 2, ...)
            mma16<BF16, kGW>(gw, n_gw, kNT, lane, [&](int r, int j) { return sH[j * sw + kt * 16 + r]; },
                             [&](int t, int j, int c) { return sE[((ch + 2 * t) * 16 + c) * se + j]; });
        }
    }

    // this work-group's partial of G_W for the block's rows
    if (has_kt) {
        const int k0 = kt * 16 + 4 * h4;
        if (k0 < Kp) {
            float *part = a.w_partial + static_cast<size_t>(tile.partial) * a.slot_rows * Kp;
#pragma unroll
            for (int t = 0; t < kGW; ++t) {
                if (t >= n_gw) break;
                const int i = (ch + 2 * t) * 16 + c16;
                *reinterpret_cast<float4 *>(part + static_cast<size_t>(i) * Kp + k0) =
                    make_float4(gw[t][0], gw[t][1], gw[t][2], gw[t][3]);
            }
        }
    }
}

// W rows of the part's dense blocks: sum the tiles' partials in tile order,
// then the Langevin step.  One thread per (row, quad).
__global__ __launch_bounds__(128) void dense_w_update_kernel(DenseIterArgs a)
{
    const int b = blockIdx.y;
    const DenseBlock blk = a.blocks[b];
    const int nq = a.Kp / 4;
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= blk.m * nq) return;
    const int i = w / nq, k0 = 4 * (w % nq);
    const IterScalars it = iter_scalars(a.clk);
    // partials loaded 32 at a time (one round trip for most blocks), added in
    // partial order
    constexpr int kBatchP = 32;
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    const float *base = a.w_partial + (static_cast<size_t>(blk.first_partial) * a.slot_rows + i) * a.Kp + k0;
    const size_t stride = static_cast<size_t>(a.slot_rows) * a.Kp;
    for (int t0 = 0; t0 < blk.n_tiles; t0 += kBatchP) {
        float4 p[kBatchP];
#pragma unroll
        for (int u = 0; u < kBatchP; ++u)   // past the last partial: the last one again, not added
            p[u] = *reinterpret_cast<const float4 *>(base + min(t0 + u, blk.n_tiles - 1) * stride);
#pragma unroll
        for (int u = 0; u < kBatchP; ++u) {
            if (t0 + u < blk.n_tiles) {
                g.x += p[u].x;
                g.y += p[u].y;
                g.z += p[u].z;
                g.w += p[u].w;
            }
        }
    }
    const float *x = a.x_old[0] + static_cast<size_t>(blk.row0 + i) * a.Kp + k0;
    const float xo[4] = {x[0], x[1], x[2], x[3]};
    const float gr[4] = {g.x, g.y, g.z, g.w};
    dense_langevin(a, it, 0, blk.row0 + i, k0, xo, gr);
}

template <bool BF16, bool VAL16>
hipError_t launch_tiles(const DenseIterArgs &a, int lik, size_t lds, hipStream_t stream)
{
    const dim3 grid(static_cast<unsigned>(a.n_tiles)), block(kDenseThreads);
    switch (lik) {
    case LIK_GAUSS: hipLaunchKernelGGL((dense_tile_kernel<BF16, LIK_GAUSS, VAL16>), grid, block, lds, stream, a); break;
    case LIK_POISSON: hipLaunchKernelGGL((dense_tile_kernel<BF16, LIK_POISSON, VAL16>), grid, block, lds, stream, a); break;
    case LIK_HALF: hipLaunchKernelGGL((dense_tile_kernel<BF16, LIK_HALF, VAL16>), grid, block, lds, stream, a); break;
    case LIK_GAMMA: hipLaunchKernelGGL((dense_tile_kernel<BF16, LIK_GAMMA, VAL16>), grid, block, lds, stream, a); break;
    default: hipLaunchKernelGGL((dense_tile_kernel<BF16, LIK_GENERAL, VAL16>), grid, block, lds, stream, a); break;
    }
    return hipGetLastError();
}

}  // namespace

size_t dense_lds_bytes(int max_m, int KS)
{
    const int MT = (max_m + 31) / 32 * 32;   // at least the padded height of any block
    return sizeof(float) * (static_cast<size_t>(MT) * (KS + 1) + static_cast<size_t>(kNT) * (KS + 1) +
                            static_cast<size_t>(MT) * (kNT + 1)) +
           64 * 16;                              // cell codes of rows 0..63
}

hipError_t launch_dense_iter(const DenseIterArgs &a, int lik, bool bf16, int max_m, hipStream_t stream)
{
    if (a.n_tiles == 0) return hipSuccess;
    const size_t lds = dense_lds_bytes(max_m, a.KS);
    // BF16 values only with BF16 operands; FP32 operands read FP32 values
    if ((a.val == nullptr) == (a.val16 == nullptr) || (a.val16 != nullptr && !bf16)) return hipErrorInvalidValue;
    hipError_t e = !bf16        ? launch_tiles<false, false>(a, lik, lds, stream)
                   : a.val16    ? launch_tiles<true, true>(a, lik, lds, stream)
                                : launch_tiles<true, false>(a, lik, lds, stream);
    if (e != hipSuccess) return e;
    const int rows_q = max_m * (a.Kp / 4);
    hipLaunchKernelGGL(dense_w_update_kernel, dim3((rows_q + 127) / 128, a.n_blocks), dim3(128), 0, stream, a);
    return hipGetLastError();
}

hipError_t dense_prepare(int max_m, int KS)
{
    const int lds = static_cast<int>(dense_lds_bytes(max_m, KS));
    const void *fns[] = {
        reinterpret_cast<const void *>(&dense_tile_kernel<false, LIK_GAUSS, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<false, LIK_POISSON, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<false, LIK_HALF, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<false, LIK_GAMMA, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<false, LIK_GENERAL, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_GAUSS, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_POISSON, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_HALF, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_GAMMA, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_GENERAL, false>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_GAUSS, true>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_POISSON, true>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_HALF, true>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_GAMMA, true>),
        reinterpret_cast<const void *>(&dense_tile_kernel<true, LIK_GENERAL, true>)};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace psgld

// ebic_kernels.hip -- gfx950 kernels of the EBIC fitness evaluation.
//
// The evaluation counts, for every individual (an ordered column list
// c_0..c_{k-1}), the rows whose values follow the >= chain along that order,
// and optionally the reversed (<=) chain (EBIC paper, Methods, "Handling
// missing values"; rows up to 2^31-1 per GPU, Methods, "Support for Big
// Data").
//
// Data layout: the resident matrix is column-major FP32 with a leading
// dimension padded to 64 rows, so the 64 rows of one wave read one column
// as a single coalesced 256-byte segment.
//
// Work decomposition of k_eval: a block owns a contiguous range of 64-row
// tiles and one group of up to P individuals. It walks its range L tiles at
// a time: the block stages those L*64 rows of every column into LDS (column
// major, so lane l of a wave reads bank l), then each wave takes every W-th
// individual of the group and evaluates it on all L sub-tiles at once: lane
// l holds row l of each sub-tile, and for each column step j a pair of
// compares is reduced across the wave with a ballot, so the running
// positive/negative masks of 64 rows live in scalar registers. A wave stops
// an individual as soon as no row of any of its L sub-tiles can still match
// (wave-uniform early exit). Per-individual counts are popcounts of the
// masks, accumulated in LDS per block and added to global memory once per
// block with integer atomics (order-independent, so results are
// deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebic_internal.h"

namespace ebic {

namespace {

constexpr int kWave = 64;
constexpr int32_t kInvalid = -1;
constexpr int kUnroll = 2;  // columns compared between two early-exit tests

// ---------------------------------------------------------------------------
// Output initialisation: matched/negative = 0 for a valid individual, -1 for
// an invalid one (length < 1, a negative or non-monotone offset, or a column
// outside [0, cols)). k_eval reads the sign to skip invalid individuals.
// ---------------------------------------------------------------------------
__global__ void k_prep(const int32_t *__restrict__ offsets, const int32_t *__restrict__ cols,
                       int32_t n, int32_t ncols, int32_t *__restrict__ matched,
                       int32_t *__restrict__ negative)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = offsets[i], e = offsets[i + 1];
    bool ok = b >= 0 && e > b;
    for (int32_t j = b; ok && j < e; ++j) {
        const int32_t c = cols[j];
        ok = c >= 0 && c < ncols;
    }
    matched[i] = ok ? 0 : kInvalid;
    if (negative) negative[i] = ok ? 0 : kInvalid;
}

__device__ __forceinline__ float subst(float v, float fill) { return v != v ? fill : v; }

// ---------------------------------------------------------------------------
// The predicate for one individual on L sub-tiles of 64 rows.
//   base:   pointer to row `lane` of sub-tile 0 of column 0 (LDS or global)
//   stride: elements between consecutive columns
//   sub:    elements between consecutive sub-tiles (64 in LDS; in global the
//           caller clamps sub-tiles past the matrix so every read is in bounds)
// Returns the matched masks M and the negative-only masks G per sub-tile.
// ---------------------------------------------------------------------------
template <int L, bool NEG, bool SUBST, int U, bool COUNT, typename Index>
__device__ __forceinline__ void eval_individual(const float *__restrict__ base, Index stride,
                                                const Index (&sub)[L],
                                                const int32_t *__restrict__ c, int32_t k,
                                                const uint64_t (&valid)[L], float fill,
                                                uint64_t (&M)[L], uint64_t (&G)[L],
                                                uint64_t &steps)
{
    uint64_t P[L], N[L];
    float prev[L];
    {
        const float *col = base + (Index)c[0] * stride;
#pragma unroll
        for (int s = 0; s < L; ++s) {
            float v = col[sub[s]];
            if (SUBST) v = subst(v, fill);
            prev[s] = v;
            // A missing first value removes the row (exclude mode). In include
            // mode no NaN reaches here, so this only drops padding rows.
            const uint64_t ok = __ballot(v == v) & valid[s];
            P[s] = ok;
            N[s] = NEG ? ok : 0ull;
        }
    }
    // Columns are taken U at a time; indices past the end are clamped to the
    // last column, whose self-comparison (v >= v, v <= v) leaves P and N
    // unchanged (a NaN there has already cleared the row). The next group's
    // indices are fetched while the current one is compared.
    const int32_t last = k - 1;
    int32_t cn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cn[u] = c[min(1 + u, last)];
    if (COUNT) steps += L;  // the first column
    for (int32_t j = 1; j < k; j += U) {
        if (COUNT) steps += U * L;
        int32_t cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cc[u] = cn[u];
        if (j + U < k) {
#pragma unroll
            for (int u = 0; u < U; ++u) cn[u] = c[min(j + U + u, last)];
        }
        float v[U][L];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float *col = base + (Index)cc[u] * stride;
#pragma unroll
            for (int s = 0; s < L; ++s) {
                v[u][s] = col[sub[s]];
                if (SUBST) v[u][s] = subst(v[u][s], fill);
            }
        }
        uint64_t alive = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int s = 0; s < L; ++s) {
                // Ordered compares: false when either side is NaN, so a missing
                // value anywhere along the chain removes the row from both trends.
                P[s] &= __ballot(v[u][s] >= prev[s]);
                if (NEG) N[s] &= __ballot(v[u][s] <= prev[s]);
                prev[s] = v[u][s];
            }
        }
#pragma unroll
        for (int s = 0; s < L; ++s) alive |= P[s] | N[s];
        if (alive == 0) break;
    }
#pragma unroll
    for (int s = 0; s < L; ++s) {
        M[s] = P[s] | N[s];
        G[s] = N[s] & ~P[s];
    }
}

// Store the per-sub-tile words of one individual with one coalesced store:
// lane s writes word s.
template <int L>
__device__ __forceinline__ void store_words(uint64_t *__restrict__ dst, const uint64_t (&w)[L],
                                            int nl, int lane)
{
    uint64_t mine = 0;
#pragma unroll
    for (int s = 0; s < L; ++s)
        if (lane == s) mine = w[s];
    if (lane < nl) dst[lane] = mine;
}

template <int L, bool NEG, int STAGE, bool SUBST, bool COUNT>
__global__ void __launch_bounds__(1024)
k_eval(EvalArgs a, const int32_t *__restrict__ offsets, const int32_t *__restrict__ colidx,
       int32_t P, int32_t n_tiles)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int T = L * kWave;
    const int lane = threadIdx.x & (kWave - 1);
    // Wave index as a scalar: every per-individual quantity derived from it
    // (CSR offsets, column indices, masks) then lives in scalar registers.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int W = blockDim.x / kWave;
    const int32_t cols = a.m.cols;

    float *tile = reinterpret_cast<float *>(smem);
    const size_t tile_elems = STAGE == STAGE_LDS ? (size_t)T * cols : 0;
    int32_t *cnt = reinterpret_cast<int32_t *>(smem + tile_elems * sizeof(float));

    const int32_t i0 = blockIdx.y * P;
    const int32_t np = min(P, a.n - i0);
    if (np <= 0) return;

    // Per-individual [matched, negative] partial counts; -1 marks invalid.
    for (int32_t t = threadIdx.x; t < np; t += blockDim.x) {
        const int32_t flag = a.matched[i0 + t] < 0 ? kInvalid : 0;
        cnt[2 * t] = flag;
        cnt[2 * t + 1] = flag;
    }

    const int64_t t_begin = (int64_t)blockIdx.x * n_tiles / gridDim.x;
    const int64_t t_end = (int64_t)(blockIdx.x + 1) * n_tiles / gridDim.x;
    const int64_t words = (a.m.rows + 63) / 64;
    const float *X = (STAGE == STAGE_DIRECT && a.m.Xfill && (a.flags & 1u)) ? a.m.Xfill : a.m.X;
    const bool include = (a.flags & 1u) != 0;

    uint64_t steps = 0;
    for (int64_t tb = t_begin; tb < t_end; tb += L) {
        const int nl = (int)min<int64_t>(L, t_end - tb);
        const int64_t row0 = tb * kWave;

        uint64_t valid[L];
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const int64_t r = row0 + s * kWave + lane;
            valid[s] = __ballot(s < nl && r < a.m.rows);
        }

        if (STAGE == STAGE_LDS) {
            __syncthreads();  // the previous chunk's readers are done
            // Stage rows [row0, row0 + nl*64) of every column, 4 rows per thread.
            const int q_per_col = nl * (kWave / 4);
            const int total = q_per_col * cols;
            const float fill = a.m.fill;
            for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
                const int c = idx / q_per_col;
                const int q = idx - c * q_per_col;
                float4 v = *reinterpret_cast<const float4 *>(X + (int64_t)c * a.m.ld + row0 + 4 * q);
                if (include) {
                    v.x = subst(v.x, fill);
                    v.y = subst(v.y, fill);
                    v.z = subst(v.z, fill);
                    v.w = subst(v.w, fill);
                }
                *reinterpret_cast<float4 *>(tile + (size_t)c * T + 4 * q) = v;
            }
            __syncthreads();
        } else {
            __syncthreads();  // cnt initialisation visible before the first update
        }

        for (int32_t ii = wave; ii < np; ii += W) {
            const int32_t i = i0 + ii;
            uint64_t M[L], G[L];
            if (cnt[2 * ii] < 0) {
#pragma unroll
                for (int s = 0; s < L; ++s) M[s] = G[s] = 0;
            } else {
                const int32_t b = offsets[i];
                const int32_t k = offsets[i + 1] - b;
                const int32_t *c = colidx + b;
                if (STAGE == STAGE_LDS) {
                    int sub[L];
#pragma unroll
                    for (int s = 0; s < L; ++s) sub[s] = s * kWave;
                    eval_individual<L, NEG, false, kUnroll, COUNT, int>(tile + lane, T, sub, c, k, valid,
                                                                        0.f, M, G, steps);
                } else {
                    // Sub-tiles past the last tile of the matrix are clamped onto
                    // it (their rows are masked out by `valid`).
                    const int64_t last = (words - 1) * kWave;
                    int64_t sub[L];
#pragma unroll
                    for (int s = 0; s < L; ++s) sub[s] = min<int64_t>(row0 + s * kWave, last) - row0;
                    eval_individual<L, NEG, SUBST, kUnroll, COUNT, int64_t>(X + row0 + lane, a.m.ld, sub,
                                                                           c, k, valid, a.m.fill,
                                                                           M, G, steps);
                }
                int32_t pm = 0, pg = 0;
#pragma unroll
                for (int s = 0; s < L; ++s) {
                    pm += __popcll(M[s]);
                    pg += __popcll(G[s]);
                }
                if (lane == 0) {
                    cnt[2 * ii] += pm;
                    cnt[2 * ii + 1] += pg;
                }
            }
            if (a.mmask) store_words<L>(a.mmask + (int64_t)i * words + tb, M, nl, lane);
            if (a.nmask) store_words<L>(a.nmask + (int64_t)i * words + tb, G, nl, lane);
        }
    }

    if (COUNT && lane == 0 && steps) atomicAdd(a.step_counter, (unsigned long long)steps);
    __syncthreads();
    for (int32_t t = threadIdx.x; t < np; t += blockDim.x) {
        const int32_t m = cnt[2 * t], g = cnt[2 * t + 1];
        if (m > 0) atomicAdd(a.matched + i0 + t, m);
        if (g > 0 && a.negative) atomicAdd(a.negative + i0 + t, g);
    }
}

// ---------------------------------------------------------------------------
// Layout: 64x64 tiles through LDS. Row-major source -> column-major
// destination with coalesced reads (along a source row) and coalesced writes
// (along a destination column). Sentinel cells become NaN.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_layout(const float *__restrict__ src, int64_t ld_src, int32_t src_col_major, int64_t nr,
         int32_t cols, int64_t r0, float *__restrict__ dst, int64_t ld, float sentinel,
         float *__restrict__ dst_fill, float fill)
{
    __shared__ float t[64][65];
    const int64_t rb = (int64_t)blockIdx.x * 64;  // first source row of the tile
    const int32_t cb = blockIdx.y * 64;            // first column of the tile
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    if (!src_col_major) {
        for (int y = ty; y < 64; y += 4) {
            const int64_t r = rb + y;
            const int32_t c = cb + tx;
            t[y][tx] = (r < nr && c < cols) ? src[r * ld_src + c] : 0.f;
        }
    } else {
        for (int y = ty; y < 64; y += 4) {
            const int64_t r = rb + tx;
            const int32_t c = cb + y;
            t[tx][y] = (r < nr && c < cols) ? src[(int64_t)c * ld_src + r] : 0.f;
        }
    }
    __syncthreads();
    for (int y = ty; y < 64; y += 4) {
        const int32_t c = cb + y;
        const int64_t r = rb + tx;
        if (c < cols && r < nr) {
            float v = t[tx][y];
            const bool missing = v != v || v == sentinel;
            if (missing) v = __builtin_nanf("");
            dst[(int64_t)c * ld + r0 + r] = v;
            if (dst_fill) dst_fill[(int64_t)c * ld + r0 + r] = missing ? fill : v;
        }
    }
}

__global__ void k_zero_pad(float *__restrict__ dst, int64_t rows, int64_t ld, int32_t cols)
{
    const int64_t pad = ld - rows;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= pad * cols) return;
    const int64_t c = idx / pad, r = rows + idx % pad;
    dst[c * ld + r] = 0.f;
}

template <int L, bool NEG, int STAGE, bool SUBST, bool COUNT>
const void *kernel_ptr()
{
    return reinterpret_cast<const void *>(&k_eval<L, NEG, STAGE, SUBST, COUNT>);
}

template <bool NEG, int STAGE, bool SUBST, bool COUNT>
const void *pick_L(int L)
{
    switch (L) {
    case 1: return kernel_ptr<1, NEG, STAGE, SUBST, COUNT>();
    case 2: return kernel_ptr<2, NEG, STAGE, SUBST, COUNT>();
    case 4: return kernel_ptr<4, NEG, STAGE, SUBST, COUNT>();
    default: return nullptr;
    }
}

template <bool COUNT>
const void *pick_variant(const LaunchCfg &cfg, bool neg, bool subst)
{
    if (cfg.staging == STAGE_LDS)
        return neg ? pick_L<true, STAGE_LDS, false, COUNT>(cfg.L)
                   : pick_L<false, STAGE_LDS, false, COUNT>(cfg.L);
    if (neg)
        return subst ? pick_L<true, STAGE_DIRECT, true, COUNT>(cfg.L)
                     : pick_L<true, STAGE_DIRECT, false, COUNT>(cfg.L);
    return subst ? pick_L<false, STAGE_DIRECT, true, COUNT>(cfg.L)
                 : pick_L<false, STAGE_DIRECT, false, COUNT>(cfg.L);
}

const void *pick_kernel(const LaunchCfg &cfg, uint32_t flags, bool has_fill_copy, bool count)
{
    const bool neg = (flags & 2u) != 0;
    const bool subst = (flags & 1u) != 0 && !has_fill_copy;
    return count ? pick_variant<true>(cfg, neg, subst) : pick_variant<false>(cfg, neg, subst);
}

}  // namespace

size_t eval_lds_bytes(const LaunchCfg &cfg, int32_t cols)
{
    size_t b = (size_t)cfg.P * 2 * sizeof(int32_t);
    if (cfg.staging == STAGE_LDS) b += (size_t)cfg.L * kWave * cols * sizeof(float);
    return b;
}

int eval_occupancy(const LaunchCfg &cfg, int32_t cols, uint32_t flags)
{
    const void *k = pick_kernel(cfg, flags, false, false);
    if (!k) return 0;
    int blocks = 0;
    const size_t lds = eval_lds_bytes(cfg, cols);
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, cfg.W * kWave, lds) != hipSuccess)
        return 0;
    return blocks;
}

hipError_t launch_eval(const EvalArgs &a, const LaunchCfg &cfg, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1)
{
    if (a.n <= 0) return hipSuccess;
    {
        const int threads = 256;
        const int blocks = (a.n + threads - 1) / threads;
        hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(threads), 0, s, a.offsets, a.cols, a.n,
                           a.m.cols, a.matched, a.negative);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const void *k = pick_kernel(cfg, a.flags, a.m.Xfill != nullptr, a.step_counter != nullptr);
    if (!k) return hipErrorInvalidValue;
    const int64_t words = (a.m.rows + 63) / 64;
    const int32_t n_tiles = (int32_t)words;
    const int32_t groups = (a.n + cfg.P - 1) / cfg.P;
    const size_t lds = eval_lds_bytes(cfg, a.m.cols);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    EvalArgs args = a;
    const int32_t *offs = a.offsets;
    const int32_t *cidx = a.cols;
    int32_t P = cfg.P;
    int32_t nt = n_tiles;
    void *params[] = {&args, &offs, &cidx, &P, &nt};
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
    e = hipLaunchKernel(k, dim3(cfg.blocks, groups), dim3(cfg.W * kWave), params, lds, s);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, s);
    return e;
}

hipError_t launch_layout(const float *src, int64_t ld_src, bool src_col_major, int64_t nr,
                         int32_t cols, int64_t r0, float *dst, int64_t ld, float sentinel,
                         float *dst_fill, float fill, hipStream_t s)
{
    if (nr <= 0) return hipSuccess;
    dim3 grid((unsigned)((nr + 63) / 64), (unsigned)((cols + 63) / 64));
    hipLaunchKernelGGL(k_layout, grid, dim3(256), 0, s, src, ld_src, (int32_t)src_col_major, nr,
                       cols, r0, dst, ld, sentinel, dst_fill, fill);
    return hipGetLastError();
}

hipError_t launch_zero_pad(float *dst, int64_t rows, int64_t ld, int32_t cols, hipStream_t s)
{
    const int64_t total = (ld - rows) * cols;
    if (total <= 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(k_zero_pad, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads),
                       0, s, dst, rows, ld, cols);
    return hipGetLastError();
}

}  // namespace ebic

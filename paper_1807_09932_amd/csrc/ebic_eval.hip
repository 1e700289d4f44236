// ebic_eval.hip -- gfx950 kernels of the EBIC fitness evaluation.
//
// The evaluation counts, for every individual (an ordered column list
// c_0..c_{k-1}), the rows whose values follow the >= chain along that order,
// and optionally the reversed (<=) chain (EBIC paper, Methods, "Handling
// missing values"; rows up to 2^31-1 per GPU, Methods, "Support for Big
// Data"). All outputs are integers decided by exact FP32 compares.
//
// Work decomposition. A work item is (a group of up to P individuals of one
// population, a contiguous range of 64-row tiles of its matrix). The block
// that owns an item walks the range L tiles at a time: it stages those
// L*64 rows of every column into LDS (column-major, so lane l of a wave
// reads bank l), then each wave takes every W-th individual of the group and
// evaluates it on the L sub-tiles together: lane l holds row l of each
// sub-tile; for each column step a pair of compares is reduced across the
// wave with a ballot, so the running positive and negative masks of 64 rows
// live in scalar registers; the individual stops as soon as no row of its
// L sub-tiles can still match (a wave-uniform early exit). Counts are
// popcounts of the masks, accumulated per block in LDS and added to global
// memory once per item with integer atomics (order-independent, so results
// are deterministic).
//
// The plain kernel (one population) launches one block per item on a 2-D
// grid. The batched kernel (many populations, many matrices) is persistent:
// its blocks take items from a device-side counter until none are left.
//
// Before either, a prep kernel validates every individual, initialises its
// outputs (0, or -1 for an invalid individual) and writes its 64-byte header
// (length, CSR start, first kWin columns clamped to the last one), which the
// evaluation reads with one scalar load per individual.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebic_internal.h"

namespace ebic {

namespace {

constexpr int32_t kInvalid = -1;

__host__ __device__ inline size_t tile_bytes_of(int32_t L, int32_t cols)
{
    return (size_t)L * kWave * cols * sizeof(float);
}

__host__ __device__ inline size_t count_bytes_of(int32_t P)
{
    return (size_t)((P + 1) & ~1) * 2 * sizeof(int32_t);
}

// ---------------------------------------------------------------------------
// Prep: validation, output initialisation and the per-individual header.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prep_one(const ReqDesc &d, int32_t i, IndHead *__restrict__ heads)
{
    const int32_t b = d.offsets[i], e = d.offsets[i + 1];
    bool ok = b >= 0 && e > b;
    for (int32_t j = b; ok && j < e; ++j) {
        const int32_t c = d.colidx[j];
        ok = c >= 0 && c < d.cols;
    }
    d.matched[i] = ok ? 0 : kInvalid;
    if (d.negative) d.negative[i] = ok ? 0 : kInvalid;
    const int32_t k = ok ? e - b : 0;
    int32_t w[kWin];
#pragma unroll
    for (int u = 0; u < kWin; ++u) w[u] = ok ? d.colidx[b + min(u, k - 1)] : 0;
    int4 *dst = reinterpret_cast<int4 *>(heads + d.head_base + i);
    dst[0] = make_int4(k, b, 0, 0);
    dst[1] = make_int4(0, 0, 0, 0);
    dst[2] = make_int4(w[0], w[1], w[2], w[3]);
    dst[3] = make_int4(w[4], w[5], w[6], w[7]);
}

__global__ void k_prep(ReqDesc d, IndHead *__restrict__ heads)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.n) prep_one(d, i, heads);
}

__global__ void k_prep_batch(BatchHeader *hdr, const ReqDesc *__restrict__ descs,
                             const int64_t *__restrict__ first, IndHead *__restrict__ heads)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) hdr->counter = 0;
    const int64_t total = hdr->total_ind;
    const int32_t nreq = hdr->n_req;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
        int32_t lo = 0, hi = nreq - 1;  // the last request with first[q] <= g
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (first[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        prep_one(descs[lo], (int32_t)(g - first[lo]), heads);
    }
}

// ---------------------------------------------------------------------------
// The predicate.
// ---------------------------------------------------------------------------

// All-ones if x > y (both wave-uniform), else zero. Produced by scalar
// instructions the compiler cannot see through, so that an exit test
// `(live & mask) == 0` stays a single 64-bit AND instead of being split
// into a second, boolean condition.
__device__ __forceinline__ uint64_t ones_if_greater(int32_t x, int32_t y)
{
    uint64_t m;
    asm volatile("s_cmp_gt_i32 %1, %2\n\ts_cselect_b64 %0, -1, 0" : "=s"(m) : "s"(x), "s"(y) : "scc");
    return m;
}

// One individual on L LDS-staged sub-tiles of 64 rows, evaluated together
// (independent loads and compares overlap their latency); the individual
// stops once no row of any sub-tile can still match. The first kWin - 1
// column steps come from the header's window, unrolled, with an exit test
// every two steps; longer individuals continue in a loop. Window entries
// past the end repeat the last column, whose self-comparison changes
// nothing (a NaN there has already cleared the row).
template <int L, bool NEG, bool COUNT>
__device__ __forceinline__ void eval_lds(const unsigned char *__restrict__ tile, const IndHead &h,
                                         const int32_t *__restrict__ colidx, int lane4,
                                         const uint64_t (&valid)[L], uint64_t (&M)[L],
                                         uint64_t (&G)[L], uint64_t &steps)
{
    constexpr int CB = L * kWave * 4;  // bytes of one staged column
    const int32_t last = h.k - 1;
    const uint64_t more2 = ones_if_greater(last, 2);
    const uint64_t more4 = ones_if_greater(last, 4);
    const uint64_t more6 = ones_if_greater(last, 6);
    const uint64_t more7 = ones_if_greater(last, 7);

    uint64_t P[L], N[L];
    float prev[L];
    {
        const unsigned char *b = tile + h.win[0] * CB + lane4;
#pragma unroll
        for (int s = 0; s < L; ++s) {
            prev[s] = *reinterpret_cast<const float *>(b + s * kWave * 4);
            // A missing first value removes the row (exclude mode); in include
            // mode no NaN is staged, so this only drops rows past the end.
            P[s] = __ballot(prev[s] == prev[s]) & valid[s];
            N[s] = NEG ? P[s] : 0ull;
        }
        if (COUNT) steps += L;
    }
    auto live = [&]() {
        uint64_t x = 0;
#pragma unroll
        for (int s = 0; s < L; ++s) x |= P[s] | N[s];
        return x;
    };
#define EBIC_STEP(col)                                                             \
    {                                                                              \
        const unsigned char *b_ = tile + (col) * CB + lane4;                       \
        _Pragma("unroll") for (int s = 0; s < L; ++s)                              \
        {                                                                          \
            const float v_ = *reinterpret_cast<const float *>(b_ + s * kWave * 4); \
            /* Ordered compares: false when either side is NaN, so a missing */   \
            /* value anywhere along the chain removes the row from both trends. */ \
            P[s] &= __ballot(v_ >= prev[s]);                                       \
            if (NEG) N[s] &= __ballot(v_ <= prev[s]);                              \
            prev[s] = v_;                                                          \
        }                                                                          \
        if (COUNT) steps += L;                                                     \
    }
    if (last == 0) goto done;
    EBIC_STEP(h.win[1]);
    EBIC_STEP(h.win[2]);
    if ((live() & more2) == 0) goto done;
    EBIC_STEP(h.win[3]);
    EBIC_STEP(h.win[4]);
    if ((live() & more4) == 0) goto done;
    EBIC_STEP(h.win[5]);
    EBIC_STEP(h.win[6]);
    if ((live() & more6) == 0) goto done;
    EBIC_STEP(h.win[7]);
    if ((live() & more7) == 0) goto done;
    for (int32_t u = kWin; u <= last; u += 2) {
        EBIC_STEP(colidx[h.begin + u]);
        EBIC_STEP(colidx[h.begin + min(u + 1, last)]);
        if (live() == 0) break;
    }
#undef EBIC_STEP
done:
#pragma unroll
    for (int s = 0; s < L; ++s) {
        M[s] = P[s] | N[s];
        G[s] = N[s] & ~P[s];
    }
}

// One individual read straight from the column-major matrix (matrices too
// wide to stage). `xr` points at row (row0 + lane) of column 0; `sub`
// holds the element offsets of the L sub-tiles (clamped by the caller so
// that every read stays inside the matrix).
template <int L, bool NEG, bool COUNT>
__device__ __forceinline__ void eval_direct(const float *__restrict__ xr, int64_t ld,
                                            const int64_t (&sub)[L], const IndHead &h,
                                            const int32_t *__restrict__ colidx, float fill,
                                            bool subst, const uint64_t (&valid)[L],
                                            uint64_t (&M)[L], uint64_t (&G)[L], uint64_t &steps)
{
    const int32_t last = h.k - 1;
    const int32_t *c = colidx + h.begin;
    auto load = [&](int32_t col, int s) {
        float v = xr[(int64_t)col * ld + sub[s]];
        if (subst) v = v != v ? fill : v;
        return v;
    };
    uint64_t P[L], N[L];
    float prev[L];
#pragma unroll
    for (int s = 0; s < L; ++s) {
        prev[s] = load(c[0], s);
        P[s] = __ballot(prev[s] == prev[s]) & valid[s];
        N[s] = NEG ? P[s] : 0ull;
    }
    if (COUNT) steps += L;
    for (int32_t u = 1; u <= last; u += 2) {
        const int32_t ca = c[u], cb = c[min(u + 1, last)];
        uint64_t x = 0;
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const float va = load(ca, s), vb = load(cb, s);
            P[s] &= __ballot(va >= prev[s]) & __ballot(vb >= va);
            if (NEG) N[s] &= __ballot(va <= prev[s]) & __ballot(vb <= va);
            prev[s] = vb;
            x |= P[s] | N[s];
        }
        if (COUNT) steps += 2 * L;
        if (x == 0) break;
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

// ---------------------------------------------------------------------------
// One work item: individuals [i0, i0 + np) of request d on tiles [t0, t1).
// `tile` and `cnt` are this block's LDS areas. Ends with a barrier, so a
// persistent block can start its next item right away.
// ---------------------------------------------------------------------------
template <int L, bool NEG, int STAGE, bool COUNT>
__device__ __forceinline__ void run_item(const ReqDesc &d, const IndHead *__restrict__ heads,
                                         int32_t i0, int32_t np, int64_t t0, int64_t t1,
                                         float *tile, int32_t *cnt, uint64_t &steps)
{
    constexpr int T = L * kWave;
    const int lane = threadIdx.x & (kWave - 1);
    // Wave index as a scalar: every per-individual quantity derived from it
    // (headers, column indices, masks) then lives in scalar registers.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int W = blockDim.x / kWave;
    const int64_t words = (d.rows + 63) / 64;
    const bool include = (d.flags & kFlagInclude) != 0;
    const IndHead *hb = heads + d.head_base + i0;

    for (int32_t t = threadIdx.x; t < 2 * np; t += blockDim.x) cnt[t] = 0;

    for (int64_t tb = t0; tb < t1; tb += L) {
        const int nl = (int)min<int64_t>(L, t1 - tb);
        const int64_t row0 = tb * kWave;
        uint64_t valid[L];
#pragma unroll
        for (int s = 0; s < L; ++s) valid[s] = __ballot(s < nl && row0 + s * kWave + lane < d.rows);

        __syncthreads();  // counts initialised; the previous chunk's readers are done
        if constexpr (STAGE == STAGE_LDS) {
            // Rows [row0, row0 + nl*64) of every column, 4 rows per thread.
            const int q_per_col = nl * (kWave / 4);
            const int total = q_per_col * d.cols;
            const float fill = d.fill;
            for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
                const int c = idx / q_per_col;
                const int q = idx - c * q_per_col;
                float4 v = *reinterpret_cast<const float4 *>(d.X + (int64_t)c * d.ld + row0 + 4 * q);
                if (include) {
                    v.x = v.x != v.x ? fill : v.x;
                    v.y = v.y != v.y ? fill : v.y;
                    v.z = v.z != v.z ? fill : v.z;
                    v.w = v.w != v.w ? fill : v.w;
                }
                *reinterpret_cast<float4 *>(tile + (size_t)c * T + 4 * q) = v;
            }
            __syncthreads();
        }

        for (int32_t ii = wave; ii < np; ii += W) {
            const IndHead h = hb[ii];
            // Materialise the whole header at once: one scalar-memory round
            // trip instead of a dependent load per field on the early-exit path.
            asm volatile("" ::"s"(h.k), "s"(h.begin), "s"(h.win[0]), "s"(h.win[1]), "s"(h.win[2]),
                         "s"(h.win[3]), "s"(h.win[4]), "s"(h.win[5]), "s"(h.win[6]), "s"(h.win[7]));
            uint64_t M[L], G[L];
            if (h.k == 0) {
#pragma unroll
                for (int s = 0; s < L; ++s) M[s] = G[s] = 0;
            } else {
                if constexpr (STAGE == STAGE_LDS) {
                    eval_lds<L, NEG, COUNT>(reinterpret_cast<const unsigned char *>(tile), h, d.colidx,
                                            lane * 4, valid, M, G, steps);
                } else {
                    // Sub-tiles past the last tile are clamped onto it (their
                    // rows are masked out by `valid`).
                    const int64_t last_row0 = (words - 1) * kWave;
                    int64_t sub[L];
#pragma unroll
                    for (int s = 0; s < L; ++s) sub[s] = min<int64_t>(row0 + s * kWave, last_row0) - row0;
                    eval_direct<L, NEG, COUNT>(d.X + row0 + lane, d.ld, sub, h, d.colidx, d.fill,
                                               (d.flags & kFlagSubst) != 0, valid, M, G, steps);
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
            const int64_t i = i0 + ii;
            if (d.mmask) store_words<L>(d.mmask + i * words + tb, M, nl, lane);
            if (d.nmask) store_words<L>(d.nmask + i * words + tb, G, nl, lane);
        }
    }

    __syncthreads();
    for (int32_t t = threadIdx.x; t < np; t += blockDim.x) {
        const int32_t m = cnt[2 * t], g = cnt[2 * t + 1];
        if (m > 0) atomicAdd(d.matched + i0 + t, m);
        if (g > 0 && d.negative) atomicAdd(d.negative + i0 + t, g);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Plain evaluation: block (x, y) = tile range x of individual group y.
// ---------------------------------------------------------------------------
template <int L, bool NEG, int STAGE, bool COUNT>
__global__ void __launch_bounds__(1024)
k_eval(ReqDesc d, const IndHead *__restrict__ heads, int32_t P, int32_t n_tiles,
       unsigned long long *step_counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const size_t tb = STAGE == STAGE_LDS ? tile_bytes_of(L, d.cols) : 0;
    float *tile = reinterpret_cast<float *>(smem);
    int32_t *cnt = reinterpret_cast<int32_t *>(smem + tb);
    const int32_t i0 = blockIdx.y * P;
    const int32_t np = min(P, d.n - i0);
    if (np <= 0) return;
    const int64_t t0 = (int64_t)blockIdx.x * n_tiles / gridDim.x;
    const int64_t t1 = (int64_t)(blockIdx.x + 1) * n_tiles / gridDim.x;
    uint64_t steps = 0;
    run_item<L, NEG, STAGE, COUNT>(d, heads, i0, np, t0, t1, tile, cnt, steps);
    if (COUNT && (threadIdx.x & (kWave - 1)) == 0 && steps)
        atomicAdd(step_counter, (unsigned long long)steps);
}

// ---------------------------------------------------------------------------
// Batched evaluation: persistent blocks take work items from the counter in
// the batch header until none are left; each item carries its request
// (matrix, population, flags, outputs).
// ---------------------------------------------------------------------------
template <int L, bool COUNT>
__global__ void __launch_bounds__(1024)
k_eval_batch(BatchHeader *hdr, const ReqDesc *__restrict__ descs, const Item *__restrict__ items,
             const IndHead *__restrict__ heads, int32_t tile_bytes,
             unsigned long long *step_counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t s_item;
    float *tile = reinterpret_cast<float *>(smem);
    int32_t *cnt = reinterpret_cast<int32_t *>(smem + tile_bytes);
    const int32_t n_items = __builtin_amdgcn_readfirstlane(hdr->n_items);
    uint64_t steps = 0;
    while (true) {
        if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(&hdr->counter, 1u);
        __syncthreads();
        const int32_t id = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();  // every wave has read s_item before thread 0 rewrites it
        if (id >= n_items) break;
        const Item it = items[id];
        const ReqDesc d = descs[it.req];
        const bool neg = (d.flags & kFlagNeg) != 0;
        if ((d.flags & kFlagDirect) == 0) {
            if (neg) run_item<L, true, STAGE_LDS, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
            else run_item<L, false, STAGE_LDS, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
        } else {
            if (neg) run_item<L, true, STAGE_DIRECT, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
            else run_item<L, false, STAGE_DIRECT, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
        }
    }
    if (COUNT && (threadIdx.x & (kWave - 1)) == 0 && steps)
        atomicAdd(step_counter, (unsigned long long)steps);
}

// ---------------------------------------------------------------------------
// Kernel selection.
// ---------------------------------------------------------------------------
template <int L, bool NEG, int STAGE, bool COUNT>
const void *eval_ptr()
{
    return reinterpret_cast<const void *>(&k_eval<L, NEG, STAGE, COUNT>);
}

template <bool NEG, int STAGE, bool COUNT>
const void *eval_pick_L(int L)
{
    switch (L) {
    case 1: return eval_ptr<1, NEG, STAGE, COUNT>();
    case 2: return eval_ptr<2, NEG, STAGE, COUNT>();
    case 4: return eval_ptr<4, NEG, STAGE, COUNT>();
    default: return nullptr;
    }
}

template <bool COUNT>
const void *eval_pick(int L, bool neg, int staging)
{
    if (staging == STAGE_LDS)
        return neg ? eval_pick_L<true, STAGE_LDS, COUNT>(L) : eval_pick_L<false, STAGE_LDS, COUNT>(L);
    return neg ? eval_pick_L<true, STAGE_DIRECT, COUNT>(L) : eval_pick_L<false, STAGE_DIRECT, COUNT>(L);
}

const void *eval_kernel(int L, uint32_t flags, int staging, bool count)
{
    const bool neg = (flags & kFlagNeg) != 0;
    return count ? eval_pick<true>(L, neg, staging) : eval_pick<false>(L, neg, staging);
}

const void *batch_kernel(int L, bool count)
{
    switch (L) {
    case 1: return count ? (const void *)&k_eval_batch<1, true> : (const void *)&k_eval_batch<1, false>;
    case 2: return count ? (const void *)&k_eval_batch<2, true> : (const void *)&k_eval_batch<2, false>;
    case 4: return count ? (const void *)&k_eval_batch<4, true> : (const void *)&k_eval_batch<4, false>;
    default: return nullptr;
    }
}

hipError_t set_lds(const void *k, size_t lds)
{
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace

size_t tile_lds_bytes(int32_t L, int32_t cols) { return tile_bytes_of(L, cols); }

size_t count_lds_bytes(int32_t P) { return count_bytes_of(P); }

int eval_occupancy(const LaunchCfg &cfg, int32_t cols, uint32_t flags)
{
    const void *k = eval_kernel(cfg.L, flags, cfg.staging, false);
    if (!k) return 0;
    const size_t lds = (cfg.staging == STAGE_LDS ? tile_bytes_of(cfg.L, cols) : 0) + count_bytes_of(cfg.P);
    int blocks = 0;
    if (set_lds(k, lds) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, cfg.W * kWave, lds) != hipSuccess)
        return 0;
    return blocks;
}

int batch_occupancy(int32_t L, int32_t W, size_t lds)
{
    const void *k = batch_kernel(L, false);
    if (!k) return 0;
    int blocks = 0;
    if (set_lds(k, lds) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, W * kWave, lds) != hipSuccess) return 0;
    return blocks;
}

hipError_t launch_eval(const ReqDesc &d, IndHead *heads, const LaunchCfg &cfg,
                       unsigned long long *step_counter, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1)
{
    if (d.n <= 0) return hipSuccess;
    {
        const int threads = 256;
        hipLaunchKernelGGL(k_prep, dim3((d.n + threads - 1) / threads), dim3(threads), 0, s, d, heads);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const void *k = eval_kernel(cfg.L, d.flags, cfg.staging, step_counter != nullptr);
    if (!k) return hipErrorInvalidValue;
    const int32_t n_tiles = (int32_t)((d.rows + 63) / 64);
    const int32_t groups = (d.n + cfg.P - 1) / cfg.P;
    const size_t lds = (cfg.staging == STAGE_LDS ? tile_bytes_of(cfg.L, d.cols) : 0) + count_bytes_of(cfg.P);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    ReqDesc dd = d;
    const IndHead *hh = heads;
    int32_t P = cfg.P, nt = n_tiles;
    unsigned long long *sc = step_counter;
    void *params[] = {&dd, &hh, &P, &nt, &sc};
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
    e = hipLaunchKernel(k, dim3(cfg.blocks, groups), dim3(cfg.W * kWave), params, lds, s);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, s);
    return e;
}

hipError_t launch_batch(BatchHeader *hdr, const ReqDesc *descs, const int64_t *first,
                        const Item *items, IndHead *heads, int32_t L, int32_t W, int32_t P,
                        size_t tile_bytes, int32_t grid, int32_t prep_blocks,
                        unsigned long long *step_counter, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1)
{
    hipLaunchKernelGGL(k_prep_batch, dim3(prep_blocks), dim3(256), 0, s, hdr, descs, first, heads);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void *k = batch_kernel(L, step_counter != nullptr);
    if (!k) return hipErrorInvalidValue;
    const size_t lds = tile_bytes + count_bytes_of(P);
    if ((e = set_lds(k, lds)) != hipSuccess) return e;
    BatchHeader *h = hdr;
    const ReqDesc *dd = descs;
    const Item *it = items;
    const IndHead *hh = heads;
    int32_t tb = (int32_t)tile_bytes;
    unsigned long long *sc = step_counter;
    void *params[] = {&h, &dd, &it, &hh, &tb, &sc};
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
    e = hipLaunchKernel(k, dim3(grid), dim3(W * kWave), params, lds, s);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, s);
    return e;
}

}  // namespace ebic

// ebic_breed.hip -- the stand-in evolutionary driver's breeding on the
// device: the next generation from the current one (CSR in device memory)
// and its matched counts, by the rules of ebic_breed.h, so that a run can
// alternate evaluation and breeding on one stream while the population
// stays in device memory. The host driver (ebic_ea_step) applies the same
// rules to the same streams: both breed the same generation.
//
// Populations of up to 1,024 (whose arrays fit LDS) are bred by one
// workgroup in one launch (k_breed_small). Larger ones take five kernels:
// fitness; the elites' order (each individual counts the ones ranking
// before it); one thread per child breeding into a slot of k_max columns;
// one block turning the lengths into offsets; one thread per child
// copying its slot into the packed CSR.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/ebic.h"
#include "ebic_breed.h"
#include "ebic_runtime_internal.h"

namespace ebic {
namespace {

constexpr int kThreads = 256;
constexpr int kLdsMaxK = 64;  // children built in LDS up to this k_max (64 KB per block)

__global__ void k_breed_fitness(int32_t n, const int32_t *__restrict__ offsets, const int32_t *__restrict__ matched,
                                double *__restrict__ f)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) f[i] = breed::fitness(matched[i], offsets[i + 1] - offsets[i]);
}

// order[r] = the individual of rank r, for r < ne (rank: higher fitness
// first, then the lower index); best, if not null, gets rank 0's index.
// Each thread counts the individuals that rank before its own over the
// whole population, read tile by tile from LDS (every lane reads the same
// element: a broadcast), without a data-dependent exit.
__global__ void __launch_bounds__(kThreads) k_breed_order(int32_t n, const double *__restrict__ f, int32_t ne,
                                                          int32_t *__restrict__ order, int32_t *__restrict__ best)
{
    constexpr int kTile = 2048;
    __shared__ double ft[kTile];
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const double fi = i < n ? f[i] : 0.0;
    int32_t r = 0;
    for (int32_t j0 = 0; j0 < n; j0 += kTile) {
        const int32_t m = min(kTile, n - j0);
        __syncthreads();
        for (int32_t j = threadIdx.x; j < m; j += blockDim.x) ft[j] = f[j0 + j];
        __syncthreads();
        for (int32_t j = 0; j < m; ++j) r += breed::ranks_before(ft[j], j0 + j, fi, i) ? 1 : 0;
    }
    if (i >= n) return;
    if (r < ne) order[r] = i;
    if (r == 0 && best) *best = i;
}

// Child c into slots[c k_max ...], its length into lens[c]. The child is
// built in LDS (element j of the block's thread t at j * blockDim + t, so
// the membership scans cost LDS reads instead of dependent global ones)
// when `in_lds`, else in its global slot directly.
__global__ void __launch_bounds__(kThreads) k_breed_children(ebic_ea_params p, int64_t generation, int32_t n,
                                 const int32_t *__restrict__ offsets, const int32_t *__restrict__ cols,
                                 const double *__restrict__ f, const int32_t *__restrict__ order,
                                 int32_t *__restrict__ slots, int32_t *__restrict__ lens, int32_t in_lds)
{
    extern __shared__ int32_t lds_child[];
    const int32_t c = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= n) return;
    int32_t *slot = slots + (int64_t)c * p.k_max;
    const breed::Strided child = in_lds ? breed::Strided{lds_child + threadIdx.x, (int32_t)blockDim.x}
                                        : breed::Strided{slot, 1};
    int32_t len;
    if (c < p.elite) {  // the elites, best first, carried over unchanged
        const int32_t e = order[c];
        len = breed::parent_len(p, offsets, e);
        for (int32_t j = 0; j < len; ++j) child[j] = cols[offsets[e] + j];
    } else {
        breed::Rng rng = breed::stream(p.seed, generation, n, c);
        breed::Strided buf = child;
        len = breed::breed_child(p, rng, n, offsets, cols, f, buf);
    }
    if (in_lds)
        for (int32_t j = 0; j < len; ++j) slot[j] = child[j];
    lens[c] = len;
}

// offsets[0] = 0, offsets[i + 1] = lens[0] + ... + lens[i]: one block; each
// thread sums a contiguous segment, the segment sums are scanned in LDS.
__global__ void __launch_bounds__(1024) k_breed_offsets(int32_t n, const int32_t *__restrict__ lens,
                                                        int32_t *__restrict__ offsets)
{
    __shared__ int32_t part[1024];
    const int32_t t = (int32_t)threadIdx.x, T = (int32_t)blockDim.x;
    const int32_t per = (n + T - 1) / T;
    const int32_t lo = min(n, t * per), hi = min(n, lo + per);
    int32_t s = 0;
    for (int32_t i = lo; i < hi; ++i) s += lens[i];
    part[t] = s;
    __syncthreads();
    for (int32_t d = 1; d < T; d <<= 1) {
        const int32_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - s;  // the sum of the segments before this one
    if (t == 0) offsets[0] = 0;
    for (int32_t i = lo; i < hi; ++i) {
        run += lens[i];
        offsets[i + 1] = run;
    }
}

__global__ void k_breed_compact(int32_t n, int32_t k_max, const int32_t *__restrict__ slots,
                                const int32_t *__restrict__ offsets, int32_t *__restrict__ cols)
{
    const int32_t c = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= n) return;
    const int32_t o = offsets[c], len = offsets[c + 1] - o;
    const int32_t *src = slots + (int64_t)c * k_max;
    for (int32_t j = 0; j < len; ++j) cols[o + j] = src[j];
}

// The whole breeding of a population of at most 1,024 in one workgroup of
// one thread per individual, everything in LDS: fitness; the rank order by
// a bitonic sort of (fitness, index) pairs (padded to a power of two with
// entries that rank last); one child per thread, built in an interleaved
// LDS array; the lengths' scan; the packed copy out. Five launches and
// their gaps become one.
__global__ void __launch_bounds__(1024) k_breed_small(ebic_ea_params p, int64_t generation, int32_t n,
                                                      const int32_t *__restrict__ offsets,
                                                      const int32_t *__restrict__ cols,
                                                      const int32_t *__restrict__ matched, int32_t n2,
                                                      int32_t *__restrict__ next_offsets,
                                                      int32_t *__restrict__ next_cols, int32_t *__restrict__ best)
{
    extern __shared__ __align__(16) unsigned char sm[];
    __shared__ int32_t part[1024];
    double *f = reinterpret_cast<double *>(sm);  // n, by individual
    double *key = f + n2;                        // n2, sorted into rank order
    int32_t *id = reinterpret_cast<int32_t *>(key + n2);
    int32_t *children = id + n2;
    const int32_t t = (int32_t)threadIdx.x, T = (int32_t)blockDim.x;
    const bool live = t < n;
    if (live) f[t] = breed::fitness(matched[t], offsets[t + 1] - offsets[t]);
    __syncthreads();
    for (int32_t i = t; i < n2; i += T) {
        key[i] = i < n ? f[i] : -HUGE_VAL;
        id[i] = i < n ? i : INT32_MAX;  // (padding ranks after every individual)
    }
    __syncthreads();
    for (int32_t k = 2; k <= n2; k <<= 1) {
        for (int32_t j = k >> 1; j > 0; j >>= 1) {
            for (int32_t i = t; i < n2; i += T) {
                const int32_t o = i ^ j;
                if (o > i) {
                    // blocks with (i & k) == 0 end in rank order, the others reversed
                    const bool first = (i & k) == 0;
                    const bool o_first = breed::ranks_before(key[o], id[o], key[i], id[i]);
                    if (o_first == first) {
                        const double kt = key[i];
                        key[i] = key[o];
                        key[o] = kt;
                        const int32_t it = id[i];
                        id[i] = id[o];
                        id[o] = it;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (t == 0 && best) *best = id[0];
    int32_t len = 0;
    const breed::Strided child{children + t, T};
    if (live) {
        if (t < p.elite) {  // the elites, best first, carried over unchanged
            const int32_t e = id[t];
            len = breed::parent_len(p, offsets, e);
            for (int32_t j = 0; j < len; ++j) child[j] = cols[offsets[e] + j];
        } else {
            breed::Rng rng = breed::stream(p.seed, generation, n, t);
            breed::Strided buf = child;
            len = breed::breed_child(p, rng, n, offsets, cols, f, buf);
        }
    }
    part[t] = len;
    __syncthreads();
    for (int32_t d = 1; d < T; d <<= 1) {
        const int32_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const int32_t end = part[t], start = end - len;
    if (t == 0) next_offsets[0] = 0;
    if (live) {
        next_offsets[t + 1] = end;
        for (int32_t j = 0; j < len; ++j) next_cols[start + j] = child[j];
    }
}

}  // namespace
}  // namespace ebic

using namespace ebic;

extern "C" ebic_status ebic_ea_breed(ebic_ctx *ctx, const ebic_ea_params *params, int64_t generation,
                                     int32_t n_ind, const int32_t *d_offsets, const int32_t *d_cols,
                                     const int32_t *d_matched, int32_t *d_next_offsets, int32_t *d_next_cols,
                                     int32_t *d_best, void *hip_stream)
{
    return guarded([&] {
        if (!ctx || !params) fail(EBIC_EINVAL, "ctx and params are required");
        const ebic_ea_params p = *params;
        if (const char *why = breed::params_error(p)) fail(EBIC_EINVAL, why);
        if (n_ind != p.pop_size) fail(EBIC_EINVAL, "n_ind must equal params->pop_size");
        if (generation < 1) fail(EBIC_EINVAL, "generation must be >= 1 (0 is the random first generation)");
        if (!d_offsets || !d_cols || !d_matched || !d_next_offsets || !d_next_cols)
            fail(EBIC_EINVAL, "d_offsets, d_cols, d_matched, d_next_offsets and d_next_cols are required");
        const hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
        const int32_t n = n_ind;
        const int32_t ne = std::max(p.elite, 1);
        DeviceGuard g(ctx->device);
        // Up to 1,024 individuals whose fitness, elite order and children
        // fit LDS: one workgroup does it all.
        const int32_t T = (n + kWave - 1) / kWave * kWave;
        int32_t n2 = 1;
        while (n2 < n) n2 <<= 1;
        const size_t small_lds = (size_t)n2 * (2 * sizeof(double) + sizeof(int32_t)) +
                                 (size_t)T * p.k_max * sizeof(int32_t);
        if (n <= 1024 && small_lds + 1024 * sizeof(int32_t) <= ctx->lds_per_block) {
            fault_point_launch(ctx, "breeding launch");
            hip_check(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_breed_small),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)small_lds),
                      "hipFuncSetAttribute");
            clear_last_error();
            hipLaunchKernelGGL(k_breed_small, dim3(1), dim3(T), small_lds, s, p, generation, n, d_offsets, d_cols,
                               d_matched, n2, d_next_offsets, d_next_cols, d_best);
            hip_check(hipGetLastError(), "breeding kernel");
            return;
        }
        // Scratch on the stream: fitness | elite order | lengths | child slots.
        const size_t f_bytes = (size_t)n * sizeof(double);
        const size_t o_bytes = ((size_t)ne * sizeof(int32_t) + 255) / 256 * 256;
        const size_t l_bytes = ((size_t)n * sizeof(int32_t) + 255) / 256 * 256;
        const size_t s_bytes = (size_t)n * p.k_max * sizeof(int32_t);
        auto *base = static_cast<unsigned char *>(stream_scratch(ctx, s, f_bytes + o_bytes + l_bytes + s_bytes));
        double *f = reinterpret_cast<double *>(base);
        int32_t *order = reinterpret_cast<int32_t *>(base + f_bytes);
        int32_t *lens = reinterpret_cast<int32_t *>(base + f_bytes + o_bytes);
        int32_t *slots = reinterpret_cast<int32_t *>(base + f_bytes + o_bytes + l_bytes);
        fault_point_launch(ctx, "breeding launch");
        const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
        clear_last_error();
        hipLaunchKernelGGL(k_breed_fitness, dim3(blocks), dim3(kThreads), 0, s, n, d_offsets, d_matched, f);
        clear_last_error();
        hipLaunchKernelGGL(k_breed_order, dim3(blocks), dim3(kThreads), 0, s, n, f, ne, order, d_best);
        const int32_t in_lds = p.k_max <= kLdsMaxK ? 1 : 0;
        clear_last_error();
        hipLaunchKernelGGL(k_breed_children, dim3(blocks), dim3(kThreads),
                           in_lds ? (size_t)kThreads * p.k_max * sizeof(int32_t) : 0, s, p, generation, n,
                           d_offsets, d_cols, f, order, slots, lens, in_lds);
        clear_last_error();
        hipLaunchKernelGGL(k_breed_offsets, dim3(1), dim3(1024), 0, s, n, lens, d_next_offsets);
        clear_last_error();
        hipLaunchKernelGGL(k_breed_compact, dim3(blocks), dim3(kThreads), 0, s, n, p.k_max, slots,
                           d_next_offsets, d_next_cols);
        hip_check(hipGetLastError(), "breeding kernels");
    });
}

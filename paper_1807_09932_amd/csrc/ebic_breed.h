// ebic_breed.h -- the breeding rules of the stand-in evolutionary driver,
// written once for the host driver (ebic_ea.cpp) and for the device
// kernels (ebic_breed.hip), so that both breed the same next generation
// from the same counts.
//
// The EBIC paper names the search only as evolutionary and driven by row
// counts (Introduction; Methods, "Handling missing values"); the rules
// below are a stand-in of the same shape: elitism, tournaments of two,
// one-point crossover, and one mutation (insert, delete, swap or
// substitute a column).
//
// Randomness: SplitMix64 (Steele, Lea & Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014), a Weyl sequence of step
// gamma through a 64-bit finaliser. Individual i of generation g (in a
// population of n) draws from its own window of 2^20 consecutive values of
// the seed's sequence, starting at position (g n + i) 2^20; since the
// state after p steps is seed + p gamma, every window is reached in O(1),
// so individuals are bred independently (one device thread each) and in
// any order, with the same results.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/ebic.h"

namespace ebic {
namespace breed {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kWindowLog2 = 20;  // draws per individual's window

struct Rng {
    uint64_t state;
    __host__ __device__ uint64_t next()
    {
        uint64_t z = (state += kGamma);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    // Uniform integer in [0, n) (n >= 1) from the high 32 bits of a draw,
    // by Lemire's multiply-and-shift with rejection ("Fast random integer
    // generation in an interval", ACM TOMACS 2019): the product x n spans
    // [0, n 2^32); its high word is the result, and draws whose low word
    // falls below 2^32 mod n are redrawn, so every result has the same
    // number of preimages. No 64-bit division (a long software routine on
    // the GPU); the 32-bit remainder is taken only when a rejection is
    // possible.
    __host__ __device__ uint32_t below(uint32_t n)
    {
        uint64_t m = (next() >> 32) * (uint64_t)n;
        uint32_t lo = (uint32_t)m;
        if (lo < n) {
            const uint32_t t = (0u - n) % n;  // 2^32 mod n
            while (lo < t) {
                m = (next() >> 32) * (uint64_t)n;
                lo = (uint32_t)m;
            }
        }
        return (uint32_t)(m >> 32);
    }
    // Uniform in [0, 1) with 53 random bits.
    __host__ __device__ double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// The stream of individual `index` of generation `generation` (0: the
// random first generation) in a population of n.
__host__ __device__ inline Rng stream(uint64_t seed, int64_t generation, int32_t n, int32_t index)
{
    const uint64_t pos = ((uint64_t)generation * (uint64_t)n + (uint64_t)index) << kWindowLog2;
    return Rng{seed + pos * kGamma};
}

// Stand-in fitness: matched rows weighted by 2^(k-2), so that longer trends
// followed by the same rows score higher; an invalid individual (matched
// -1) scores -inf.
__host__ __device__ inline double fitness(int32_t matched, int32_t k)
{
    if (matched < 0) return -HUGE_VAL;
    if (matched == 0) return 0.0;  // (never 0 x inf, whatever the length)
    return (double)matched * ldexp(1.0, k - 2);
}

// Rank order: higher fitness first, then the lower index (individual a
// of fitness fa before individual b of fitness fb).
__host__ __device__ inline bool ranks_before(double fa, int32_t a, double fb, int32_t b)
{
    return fa > fb || (fa == fb && a < b);
}

// The functions below take the individual being built as any indexable
// buffer (a host array, or a device thread's column of an interleaved LDS
// array); the parents are plain arrays.
template <class Buf>
__host__ __device__ inline bool contains(const Buf &ind, int32_t len, int32_t c)
{
    for (int32_t j = 0; j < len; ++j)
        if (ind[j] == c) return true;
    return false;
}

// A column of [0, n_cols) not in ind[0, len) (callers ensure one exists).
template <class Buf>
__host__ __device__ inline int32_t unused_column(Rng &rng, int32_t n_cols, const Buf &ind, int32_t len)
{
    int32_t c;
    do c = (int32_t)rng.below((uint32_t)n_cols);
    while (contains(ind, len, c));
    return c;
}

// A random individual of distinct columns, k_min..k_max long, into out
// (capacity k_max); returns its length.
template <class Buf>
__host__ __device__ inline int32_t random_individual(const ebic_ea_params &p, Rng &rng, Buf &out)
{
    const int32_t k = p.k_min + (int32_t)rng.below((uint32_t)(p.k_max - p.k_min + 1));
    int32_t len = 0;
    while (len < k) {
        out[len] = unused_column(rng, p.n_cols, out, len);
        ++len;
    }
    return len;
}

// One mutation of ind[0, k) in place (capacity k_max); returns the new
// length. The operation is drawn first; one that does not apply to this
// individual falls through to substitution.
template <class Buf>
__host__ __device__ inline int32_t mutate(const ebic_ea_params &p, Rng &rng, Buf &ind, int32_t k)
{
    const bool can_insert = k < p.k_max && k < p.n_cols;
    const bool can_delete = k > p.k_min;
    const bool can_swap = k >= 2;
    const bool can_subst = k < p.n_cols;
    const uint32_t op = rng.below(4);
    if (op == 0 && can_insert) {
        const int32_t c = unused_column(rng, p.n_cols, ind, k);
        const int32_t at = (int32_t)rng.below((uint32_t)k + 1);
        for (int32_t j = k; j > at; --j) ind[j] = ind[j - 1];
        ind[at] = c;
        return k + 1;
    }
    if (op == 1 && can_delete) {
        const int32_t at = (int32_t)rng.below((uint32_t)k);
        for (int32_t j = at; j + 1 < k; ++j) ind[j] = ind[j + 1];
        return k - 1;
    }
    if (op == 2 && can_swap) {
        const uint32_t a = rng.below((uint32_t)k), b = rng.below((uint32_t)k);
        const int32_t t = ind[a];
        ind[a] = ind[b];
        ind[b] = t;
        return k;
    }
    if (can_subst) {
        const int32_t c = unused_column(rng, p.n_cols, ind, k);
        ind[rng.below((uint32_t)k)] = c;
    }
    return k;
}

// One-point crossover: a prefix of a, then b from a random point on,
// skipping columns already present, cut to k_max and topped up to k_min
// with unused columns. Parents are at least one column long.
template <class Buf>
__host__ __device__ inline int32_t crossover(const ebic_ea_params &p, Rng &rng, const int32_t *a, int32_t ka,
                                             const int32_t *b, int32_t kb, Buf &child)
{
    const uint32_t cut = ka > 1 ? 1 + rng.below((uint32_t)ka - 1) : 1;
    const uint32_t from = rng.below((uint32_t)kb);
    int32_t len = 0;
    for (int32_t j = 0; j < (int32_t)cut && j < ka && len < p.k_max; ++j) child[len++] = a[j];
    for (int32_t j = (int32_t)from; j < kb && len < p.k_max; ++j)
        if (!contains(child, len, b[j])) child[len++] = b[j];
    while (len < p.k_min) {
        child[len] = unused_column(rng, p.n_cols, child, len);
        ++len;
    }
    return len;
}

// A parent's columns as breeding reads them: at most k_max of them (a
// caller-made population may hold longer individuals).
__host__ __device__ inline int32_t parent_len(const ebic_ea_params &p, const int32_t *offsets, int32_t i)
{
    const int32_t k = offsets[i + 1] - offsets[i];
    return k < p.k_max ? k : p.k_max;
}

// One child that is not an elite: the winner a of a tournament of two
// (ties to the lower index; a column-less parent is replaced by a random
// individual), then with probability p_crossover a crossover with the
// winner of a second tournament, then with probability p_mutation one
// mutation. Writes the child to `child` (capacity k_max), returns its
// length.
template <class Buf>
__host__ __device__ inline int32_t breed_child(const ebic_ea_params &p, Rng &rng, int32_t n,
                                               const int32_t *offsets, const int32_t *cols, const double *f,
                                               Buf &child)
{
    auto tournament = [&]() -> int32_t {
        const int32_t a = (int32_t)rng.below((uint32_t)n), b = (int32_t)rng.below((uint32_t)n);
        return f[a] > f[b] || (f[a] == f[b] && a <= b) ? a : b;
    };
    const int32_t a = tournament();
    const int32_t ka = parent_len(p, offsets, a);
    int32_t len;
    if (rng.uniform() < p.p_crossover) {
        const int32_t b = tournament();
        const int32_t kb = parent_len(p, offsets, b);
        if (ka > 0 && kb > 0) len = crossover(p, rng, cols + offsets[a], ka, cols + offsets[b], kb, child);
        else len = random_individual(p, rng, child);
    } else if (ka > 0) {
        for (int32_t j = 0; j < ka; ++j) child[j] = cols[offsets[a] + j];
        len = ka;
    } else {
        len = random_individual(p, rng, child);
    }
    if (rng.uniform() < p.p_mutation) len = mutate(p, rng, child, len);
    return len;
}

// Element j of one thread's buffer in an array interleaved over `stride`
// threads (element j of thread t at j * stride + t: consecutive threads hit
// consecutive LDS banks).
struct Strided {
    int32_t *base;
    int32_t stride;
    __host__ __device__ int32_t &operator[](int32_t j) const { return base[(int64_t)j * stride]; }
};

// Why a parameter set cannot drive a run (NULL if it can).
inline const char *params_error(const ebic_ea_params &p)
{
    if (p.n_cols < 1 || p.pop_size < 2 || p.k_min < 1 || p.k_max < p.k_min || p.k_max > p.n_cols)
        return "need n_cols >= 1, pop_size >= 2, 1 <= k_min <= k_max <= n_cols";
    if (p.elite < 0 || p.elite >= p.pop_size) return "elite must be in [0, pop_size)";
    if (!(p.p_crossover >= 0 && p.p_crossover <= 1 && p.p_mutation >= 0 && p.p_mutation <= 1))
        return "probabilities must be in [0, 1]";
    if ((int64_t)p.pop_size * p.k_max > INT32_MAX) return "pop_size x k_max must fit int32 offsets";
    return nullptr;
}

}  // namespace breed
}  // namespace ebic

// ebic_ea.cpp -- a stand-in evolutionary driver around the fitness
// evaluation: it holds a population of ordered column lists, turns the
// counts of one generation into fitness, and breeds the next generation.
//
// The EBIC paper describes the method's search only as evolutionary and
// driven by counting rows (Introduction; Methods, "Handling missing
// values"); its actual operators and fitness formula are not given there.
// The operators below are therefore a stand-in with the same shape of work
// -- mutation (insert, delete, swap, substitute a column), one-point
// crossover, tournament selection with elitism -- so that the evaluation can
// be driven generation after generation, on the host, at native speed.
//
// Every random choice comes from a counter-based generator (SplitMix64 of
// seed + counter), so a run is a pure function of its parameters and of the
// counts it is given.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_runtime_internal.h"

namespace {

// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): a Weyl sequence through a 64-bit finaliser.
struct Rng {
    uint64_t state;
    uint64_t next()
    {
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    // Uniform integer in [0, n) (n >= 1), by rejection (no modulo bias).
    uint32_t below(uint32_t n)
    {
        const uint64_t lim = UINT64_MAX - UINT64_MAX % n;
        uint64_t x;
        do x = next();
        while (x >= lim);
        return (uint32_t)(x % n);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

using Ind = std::vector<int32_t>;

}  // namespace

struct ebic_ea {
    ebic_ea_params p{};
    Rng rng{0};
    std::vector<Ind> pop;
    std::vector<int32_t> offsets, cols;  // CSR of `pop`
    std::vector<uint8_t> used;           // scratch: column membership
    int64_t generation = 0;
    int32_t best = -1;
    double best_fitness = -INFINITY;
};

namespace {

void rebuild_csr(ebic_ea *ea)
{
    ea->offsets.assign(1, 0);
    ea->cols.clear();
    for (auto &ind : ea->pop) {
        ea->cols.insert(ea->cols.end(), ind.begin(), ind.end());
        ea->offsets.push_back((int32_t)ea->cols.size());
    }
}

// A column not in `ind` (ind.size() < n_cols).
int32_t unused_column(ebic_ea *ea, const Ind &ind)
{
    for (int32_t c : ind) ea->used[c] = 1;
    int32_t c;
    do c = (int32_t)ea->rng.below((uint32_t)ea->p.n_cols);
    while (ea->used[c]);
    for (int32_t x : ind) ea->used[x] = 0;
    return c;
}

Ind random_individual(ebic_ea *ea)
{
    const int32_t k = ea->p.k_min + (int32_t)ea->rng.below((uint32_t)(ea->p.k_max - ea->p.k_min + 1));
    Ind ind;
    ind.reserve(k);
    while ((int32_t)ind.size() < k) ind.push_back(unused_column(ea, ind));
    return ind;
}

void mutate(ebic_ea *ea, Ind &ind)
{
    const int32_t k = (int32_t)ind.size();
    const bool can_insert = k < ea->p.k_max && k < ea->p.n_cols;
    const bool can_delete = k > ea->p.k_min;
    const bool can_swap = k >= 2;
    const bool can_subst = k < ea->p.n_cols;
    const uint32_t op = ea->rng.below(4);
    if (op == 0 && can_insert) {
        const int32_t c = unused_column(ea, ind);
        ind.insert(ind.begin() + ea->rng.below((uint32_t)k + 1), c);
    } else if (op == 1 && can_delete) {
        ind.erase(ind.begin() + ea->rng.below((uint32_t)k));
    } else if (op == 2 && can_swap) {
        const uint32_t a = ea->rng.below((uint32_t)k), b = ea->rng.below((uint32_t)k);
        std::swap(ind[a], ind[b]);
    } else if (can_subst) {
        const int32_t c = unused_column(ea, ind);
        ind[ea->rng.below((uint32_t)k)] = c;
    }
}

// One-point crossover: a prefix of `a`, then `b` from a random point on,
// skipping columns already present, cut to k_max and topped up to k_min.
Ind crossover(ebic_ea *ea, const Ind &a, const Ind &b)
{
    const uint32_t cut = a.size() > 1 ? 1 + ea->rng.below((uint32_t)a.size() - 1) : 1;
    const uint32_t from = ea->rng.below((uint32_t)b.size());
    Ind child(a.begin(), a.begin() + std::min<size_t>(cut, a.size()));
    for (int32_t c : child) ea->used[c] = 1;
    for (size_t j = from; j < b.size() && (int32_t)child.size() < ea->p.k_max; ++j)
        if (!ea->used[b[j]]) {
            ea->used[b[j]] = 1;
            child.push_back(b[j]);
        }
    for (int32_t c : child) ea->used[c] = 0;
    while ((int32_t)child.size() < ea->p.k_min) child.push_back(unused_column(ea, child));
    return child;
}

// Stand-in fitness: matched rows weighted by 2^(k-2), so that longer trends
// followed by the same rows score higher; invalid individuals score -inf.
double fitness(int32_t matched, size_t k)
{
    if (matched < 0) return -INFINITY;
    return (double)matched * std::ldexp(1.0, (int)k - 2);
}

}  // namespace

using namespace ebic;

extern "C" {

ebic_status ebic_ea_create(const ebic_ea_params *params, ebic_ea **out)
{
    return guarded([&] {
        if (!params || !out) fail(EBIC_EINVAL, "params and out are required");
        *out = nullptr;
        const ebic_ea_params &p = *params;
        if (p.n_cols < 1 || p.pop_size < 2 || p.k_min < 1 || p.k_max < p.k_min || p.k_max > p.n_cols)
            fail(EBIC_EINVAL, "need n_cols >= 1, pop_size >= 2, 1 <= k_min <= k_max <= n_cols");
        if (p.elite < 0 || p.elite >= p.pop_size) fail(EBIC_EINVAL, "elite must be in [0, pop_size)");
        if (!(p.p_crossover >= 0 && p.p_crossover <= 1 && p.p_mutation >= 0 && p.p_mutation <= 1))
            fail(EBIC_EINVAL, "probabilities must be in [0, 1]");
        auto ea = std::make_unique<ebic_ea>();
        ea->p = p;
        ea->rng.state = p.seed;
        ea->used.assign((size_t)p.n_cols, 0);
        ea->pop.reserve((size_t)p.pop_size);
        for (int32_t i = 0; i < p.pop_size; ++i) ea->pop.push_back(random_individual(ea.get()));
        rebuild_csr(ea.get());
        *out = ea.release();
    });
}

ebic_status ebic_ea_destroy(ebic_ea *ea)
{
    delete ea;
    return EBIC_OK;
}

ebic_status ebic_ea_population(ebic_ea *ea, const int32_t **offsets, const int32_t **cols, int32_t *n_ind,
                               int64_t *generation)
{
    return guarded([&] {
        if (!ea) fail(EBIC_EINVAL, "ea is NULL");
        if (offsets) *offsets = ea->offsets.data();
        if (cols) *cols = ea->cols.data();
        if (n_ind) *n_ind = (int32_t)ea->pop.size();
        if (generation) *generation = ea->generation;
    });
}

ebic_status ebic_ea_step(ebic_ea *ea, const int32_t *matched, int32_t *best_index, double *best_fitness)
{
    return guarded([&] {
        if (!ea || !matched) fail(EBIC_EINVAL, "ea and matched are required");
        const int32_t n = (int32_t)ea->pop.size();
        std::vector<double> f((size_t)n);
        for (int32_t i = 0; i < n; ++i) f[i] = fitness(matched[i], ea->pop[i].size());
        // Rank: fitness descending, index ascending on ties.
        std::vector<int32_t> order((size_t)n);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return f[a] > f[b]; });
        ea->best = order[0];
        ea->best_fitness = f[order[0]];
        if (best_index) *best_index = ea->best;
        if (best_fitness) *best_fitness = ea->best_fitness;
        auto tournament = [&]() -> const Ind & {
            const int32_t a = (int32_t)ea->rng.below((uint32_t)n), b = (int32_t)ea->rng.below((uint32_t)n);
            const bool pick_a = f[a] > f[b] || (f[a] == f[b] && a <= b);
            return ea->pop[pick_a ? a : b];
        };
        std::vector<Ind> next;
        next.reserve((size_t)n);
        for (int32_t e = 0; e < ea->p.elite; ++e) next.push_back(ea->pop[order[e]]);
        while ((int32_t)next.size() < n) {
            const Ind &a = tournament();
            Ind child;
            if (ea->rng.uniform() < ea->p.p_crossover) child = crossover(ea, a, tournament());
            else child = a;
            if (ea->rng.uniform() < ea->p.p_mutation) mutate(ea, child);
            next.push_back(std::move(child));
        }
        ea->pop.swap(next);
        ++ea->generation;
        rebuild_csr(ea);
    });
}

}  // extern "C"

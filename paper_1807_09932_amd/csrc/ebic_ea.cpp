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
// The breeding rules live in ebic_breed.h, shared with the device kernels
// of ebic_ea_breed: every individual draws from its own window of the
// seed's SplitMix64 sequence, so a run is a pure function of its
// parameters and of the counts it is given, wherever it is bred.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_breed.h"
#include "ebic_runtime_internal.h"

struct ebic_ea {
    ebic_ea_params p{};
    std::vector<int32_t> offsets, cols;  // the current generation, CSR
    int64_t generation = 0;
    int32_t best = -1;
    double best_fitness = -INFINITY;
};

using namespace ebic;

extern "C" {

ebic_status ebic_ea_create(const ebic_ea_params *params, ebic_ea **out)
{
    return guarded([&] {
        if (!params || !out) fail(EBIC_EINVAL, "params and out are required");
        *out = nullptr;
        const ebic_ea_params &p = *params;
        if (const char *why = breed::params_error(p)) fail(EBIC_EINVAL, why);
        auto ea = std::make_unique<ebic_ea>();
        ea->p = p;
        ea->offsets.assign(1, 0);
        std::vector<int32_t> ind((size_t)p.k_max);
        for (int32_t i = 0; i < p.pop_size; ++i) {
            breed::Rng rng = breed::stream(p.seed, 0, p.pop_size, i);
            int32_t *buf = ind.data();
            const int32_t k = breed::random_individual(p, rng, buf);
            ea->cols.insert(ea->cols.end(), ind.begin(), ind.begin() + k);
            ea->offsets.push_back((int32_t)ea->cols.size());
        }
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
        if (n_ind) *n_ind = ea->p.pop_size;
        if (generation) *generation = ea->generation;
    });
}

ebic_status ebic_ea_step(ebic_ea *ea, const int32_t *matched, int32_t *best_index, double *best_fitness)
{
    return guarded([&] {
        if (!ea || !matched) fail(EBIC_EINVAL, "ea and matched are required");
        const ebic_ea_params &p = ea->p;
        const int32_t n = p.pop_size;
        std::vector<double> f((size_t)n);
        for (int32_t i = 0; i < n; ++i) f[i] = breed::fitness(matched[i], ea->offsets[i + 1] - ea->offsets[i]);
        // Rank: fitness descending, index ascending on ties.
        std::vector<int32_t> order((size_t)n);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(),
                  [&](int32_t a, int32_t b) { return breed::ranks_before(f[a], a, f[b], b); });
        ea->best = order[0];
        ea->best_fitness = f[order[0]];
        if (best_index) *best_index = ea->best;
        if (best_fitness) *best_fitness = ea->best_fitness;
        const int64_t g = ea->generation + 1;
        std::vector<int32_t> offs(1, 0), cols, child((size_t)p.k_max);
        cols.reserve(ea->cols.size());
        for (int32_t c = 0; c < n; ++c) {
            int32_t len;
            if (c < p.elite) {  // the elites, best first, carried over unchanged
                const int32_t e = order[c];
                len = breed::parent_len(p, ea->offsets.data(), e);
                std::copy_n(ea->cols.begin() + ea->offsets[e], len, child.begin());
            } else {
                breed::Rng rng = breed::stream(p.seed, g, n, c);
                int32_t *buf = child.data();
                len = breed::breed_child(p, rng, n, ea->offsets.data(), ea->cols.data(), f.data(), buf);
            }
            cols.insert(cols.end(), child.begin(), child.begin() + len);
            offs.push_back((int32_t)cols.size());
        }
        ea->offsets.swap(offs);
        ea->cols.swap(cols);
        ea->generation = g;
    });
}

}  // extern "C"

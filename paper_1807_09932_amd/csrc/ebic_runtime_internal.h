// ebic_runtime_internal.h -- the context object and helpers shared by the
// runtime translation units. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ebic_internal.h"

namespace ebic {

struct Matrix {
    DevMatrix dev;
    float *X = nullptr;
    float *Xfill = nullptr;
    size_t bytes = 0;
    float sentinel = 0.f;
};

// Shape class of a tuning entry: log2 buckets of rows, columns, population
// size and mean individual length.
struct TuneKey {
    int32_t rows_b, cols_b, n_b, k_b;
    bool operator<(const TuneKey &o) const
    {
        if (rows_b != o.rows_b) return rows_b < o.rows_b;
        if (cols_b != o.cols_b) return cols_b < o.cols_b;
        if (n_b != o.n_b) return n_b < o.n_b;
        return k_b < o.k_b;
    }
};

struct BatchState;  // ebic_batch.cpp

}  // namespace ebic

struct ebic_ctx {
    int device = 0;
    int cu_count = 0;
    size_t lds_per_block = 65536;
    size_t lds_per_cu = 65536;
    std::string arch;
    std::mutex mu;
    void *(*alloc)(size_t, void *) = nullptr;
    void (*release)(void *, void *) = nullptr;
    void *alloc_user = nullptr;
    std::map<int32_t, ebic::Matrix> matrices;
    int32_t next_matrix = 0;
    ebic::LaunchCfg override_cfg;              // W > 0: forced launch shape
    std::map<ebic::TuneKey, ebic::LaunchCfg> tuned;
    ebic::BatchState *batch = nullptr;
    bool batch_state_allocated = false;
    // Diagnostics (ebic_set_profiling / ebic_read_profile).
    int32_t prof_mode = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    unsigned long long *d_step_counter = nullptr;
};

namespace ebic {

void *ctx_alloc(ebic_ctx *ctx, size_t bytes);
void ctx_free(ebic_ctx *ctx, void *p);
const Matrix &ctx_matrix(ebic_ctx *ctx, int32_t id);
LaunchCfg plan_eval(ebic_ctx *ctx, const Matrix &m, int32_t n, int64_t nnz, uint32_t flags);
// Launch one evaluation with the context's diagnostics applied.
hipError_t ctx_launch_eval(ebic_ctx *ctx, EvalArgs a, const LaunchCfg &cfg, hipStream_t s);

// ebic_tune.cpp
TuneKey tune_key(int64_t rows, int32_t cols, int32_t n, int64_t nnz);
LaunchCfg tuned_cfg(ebic_ctx *ctx, int64_t rows, int32_t cols, int32_t n, int64_t nnz);
LaunchCfg default_cfg(int64_t rows, int32_t cols, int32_t n);
void load_tune_cache(ebic_ctx *ctx, const std::string &path);

// ebic_batch.cpp
void destroy_batch_state(ebic_ctx *ctx);

}  // namespace ebic

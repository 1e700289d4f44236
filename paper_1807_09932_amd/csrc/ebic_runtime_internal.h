// ebic_runtime_internal.h -- the context object and helpers shared by the
// runtime translation units. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_internal.h"

namespace ebic {

struct Matrix {
    DevMatrix dev;
    float *X = nullptr;
    float *Xfill = nullptr;
    uint16_t *C = nullptr;      // rank codes of X (cols <= kMaxCodeCols)
    uint16_t *Cfill = nullptr;  // rank codes of Xfill
    uint8_t *B = nullptr;       // byte rank codes (cols <= kMaxByteCols)
    uint8_t *Hc = nullptr;      // 16-bit rank codes (kMaxByteCols < cols <= kMaxCodeCols)
    size_t bytes = 0;        // everything resident for this matrix
    size_t value_bytes = 0;  // X and Xfill
    float sentinel = 0.f;
    int32_t has_missing = -1;  // from the SWAR code build (-1: not built)
    double upload_ms = 0;
};

// Shape class of a tuning entry: log2 buckets of rows, columns, population
// size and mean individual length.
struct TuneKey {
    int32_t kind;  // 0: one population, 1: a batch
    int32_t rows_b, cols_b, n_b, k_b;
    bool operator<(const TuneKey &o) const
    {
        if (kind != o.kind) return kind < o.kind;
        if (rows_b != o.rows_b) return rows_b < o.rows_b;
        if (cols_b != o.cols_b) return cols_b < o.cols_b;
        if (n_b != o.n_b) return n_b < o.n_b;
        return k_b < o.k_b;
    }
};

struct BatchState;  // ebic_batch.cpp

// Device scratch owned by the context, one per stream: work on one stream
// runs in order, so consecutive calls on it can reuse the same buffer.
struct Scratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};

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
    int64_t graph_captures = 0;  // batch graphs captured so far (under mu)
    std::mutex batch_mu;  // guards the batch graph cache (captures run outside it)
    bool batch_state_allocated = false;
    std::map<hipStream_t, ebic::Scratch> scratch;
    // Diagnostics (ebic_set_profiling / ebic_read_profile).
    int32_t prof_mode = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    unsigned long long *d_step_counter = nullptr;
};

namespace ebic {

// Errors: thrown inside the library, turned into an ebic_status (and the
// thread's last-error message) at the ABI boundary by guarded().
struct Error : std::runtime_error {
    ebic_status code;
    Error(ebic_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(ebic_status code, const std::string &msg) { throw Error(code, msg); }

inline void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) fail(EBIC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void set_last_error(const std::string &msg);

template <typename F>
ebic_status guarded(F &&f)
{
    try {
        set_last_error("");
        f();
        return EBIC_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return EBIC_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return EBIC_EINVAL;
    } catch (...) {
        set_last_error("unknown error");
        return EBIC_EINVAL;
    }
}

// Makes the context's device current for the duration of a call and
// restores the caller's device afterwards.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        hip_check(hipGetDevice(&prev), "hipGetDevice");
        if (prev != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;
};

void *ctx_alloc(ebic_ctx *ctx, size_t bytes);
void ctx_free(ebic_ctx *ctx, void *p);
const Matrix &ctx_matrix(ebic_ctx *ctx, int32_t id);
LaunchCfg plan_eval(ebic_ctx *ctx, const Matrix &m, int32_t n, int64_t nnz, uint32_t flags);
// The kernels' view of one request; `staging` decides whether include mode
// reads the fill copy or substitutes on the fly.
ReqDesc make_desc(const Matrix &m, int32_t n, const int32_t *offsets, const int32_t *cols,
                  uint32_t flags, int32_t *matched, int32_t *negative, uint64_t *mmask,
                  uint64_t *nmask, int32_t staging);
// At least `bytes` of device scratch private to stream `s` (grown on demand;
// a grown buffer replaces the old one after the stream has drained).
void *stream_scratch(ebic_ctx *ctx, hipStream_t s, size_t bytes);
// Launch one evaluation with the context's diagnostics applied.
hipError_t ctx_launch_eval(ebic_ctx *ctx, const ReqDesc &d, const LaunchCfg &cfg, hipStream_t s);

// ebic_tune.cpp
TuneKey tune_key(int64_t rows, int32_t cols, int32_t n, int64_t nnz);
LaunchCfg tuned_cfg(ebic_ctx *ctx, int64_t rows, int32_t cols, int32_t n, int64_t nnz);
LaunchCfg tuned_batch_cfg(ebic_ctx *ctx, int64_t total_ind, int64_t mean_rows, int32_t max_cols,
                          int64_t nnz);
LaunchCfg default_batch_cfg(int32_t max_cols);
LaunchCfg default_cfg(int64_t rows, int32_t cols, int32_t n);
void load_tune_cache(ebic_ctx *ctx, const std::string &path);

// ebic_batch.cpp
void destroy_batch_state(ebic_ctx *ctx);

}  // namespace ebic

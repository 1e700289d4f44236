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
    uint8_t *T10 = nullptr;     // 10-bit rank codes (kMaxByteCols < cols <= kMaxT10Cols)
    uint32_t *Gx = nullptr;     // pairwise order bitmaps of X (built on first use)
    uint32_t *Gf = nullptr;     // of the fill-substituted values (include mode, cells missing)
    size_t bytes = 0;        // everything resident for this matrix
    size_t value_bytes = 0;  // X and Xfill
    float sentinel = 0.f;
    int32_t has_missing = -1;  // from the SWAR code build (-1: not built)
    bool pairs_failed = false;  // a build of the pair bitmaps found no memory: not tried again
    double upload_ms = 0;
    // Holders that keep the matrix from being released (under ctx->mu):
    // calls between planning and enqueuing, and serving requests from
    // submission to completion.
    int32_t refs = 0;
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

// Host-side fault injection plan (see parse_fault_plan).
struct FaultPlan {
    int64_t alloc_after = -1;   // -1: off
    int64_t launch_after = -1;
};

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
    // Fault injection (tests of the error paths; see FaultPlan).
    // Pinned host staging of uploads (two buffers used alternately, and the
    // events of the copies that last read them; under mu).
    void *up_pin[2] = {nullptr, nullptr};
    hipEvent_t up_done[2] = {nullptr, nullptr};
    size_t up_pin_bytes = 0;
    std::mutex fault_mu;
    ebic::FaultPlan fault;
    int64_t allocs_done = 0, launches_done = 0;
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

// References that keep matrices resident while a call or a serving request
// uses them. matrix_ref_locked takes one (the caller holds ctx->mu; fails
// with EBIC_ENOENT for an unknown handle); matrix_unref drops one (takes
// ctx->mu itself).
void matrix_ref_locked(ebic_ctx *ctx, int32_t id);
void matrix_unref(ebic_ctx *ctx, int32_t id);

// The references of one call, dropped when it goes out of scope (after the
// call's work has been enqueued, or on an error).
class MatrixHold {
  public:
    explicit MatrixHold(ebic_ctx *ctx) : ctx_(ctx) {}
    ~MatrixHold()
    {
        for (int32_t id : ids_) matrix_unref(ctx_, id);
    }
    void add_locked(int32_t id)
    {
        matrix_ref_locked(ctx_, id);
        ids_.push_back(id);
    }
    MatrixHold(const MatrixHold &) = delete;
    MatrixHold &operator=(const MatrixHold &) = delete;

  private:
    ebic_ctx *ctx_;
    std::vector<int32_t> ids_;
};

// Host-side fault injection for tests of the error paths (environment
// variable EBIC_FAULT, read at ebic_create): "alloc" or "alloc:N" makes
// the device allocation after N successful ones fail with EBIC_ENOMEM,
// "launch" or "launch:N" makes the kernel launch after N successful ones
// fail with EBIC_EHIP, both before anything is enqueued; a comma separates
// both. Each fault fires once.
FaultPlan parse_fault_plan(const char *spec);
// Throws the injected launch failure when it is due (the launch wrappers
// call it before enqueuing).
void fault_point_launch(ebic_ctx *ctx, const char *what);

// Diagnostics on stderr at the level of EBIC_LOG (read at ebic_create):
// 0 off (default), 1 errors returned by the ABI, 2 also uploads, releases
// and serving-engine events, 3 also every launch plan.
int log_level();
void log_msg(int level, const std::string &msg);

void *ctx_alloc(ebic_ctx *ctx, size_t bytes);
void ctx_free(ebic_ctx *ctx, void *p);
const Matrix &ctx_matrix(ebic_ctx *ctx, int32_t id);
Matrix &ctx_matrix_mut(ebic_ctx *ctx, int32_t id);

// FP16 rank codes are built on first use (a forced or tuned shape that
// stages them), except those exclude mode needs on a matrix with missing
// cells, which the upload builds. What a planner may do about absent codes:
enum CodesMode {
    CODES_EXISTING = 0,  // plan with what is resident (no allocation)
    CODES_BUILD = 1,     // build the codes a plan stages, then plan with them
    CODES_REPORT = 2,    // plan as if buildable codes existed (build nothing)
};
// Whether the FP16 codes of a mode can exist (include mode codes the fill
// copy, which must be kept).
bool codes_buildable(const Matrix &m, bool include);
// Build them now (under ctx->mu): allocation, the codes kernel on a private
// stream, and a wait for it.
void build_fp16_codes(ebic_ctx *ctx, Matrix &m, bool include);
// 16-bit SWAR codes (129..384 columns) are built on first use too: whether
// they can serve a mode, and their build (under ctx->mu).
bool halves_buildable(const Matrix &m, bool include);
void build_half_codes(ebic_ctx *ctx, Matrix &m);
bool pairs_buildable(const Matrix &m);
void build_pairs(ebic_ctx *ctx, Matrix &m, bool include);
const uint32_t *pairs_for(const Matrix &m, bool include);  // the bitmaps a mode reads, or null
LaunchCfg plan_eval(ebic_ctx *ctx, Matrix &m, int32_t n, int64_t nnz, uint32_t flags,
                    CodesMode codes = CODES_BUILD, bool masks = false);
// The kernels' view of one request; `staging` decides whether include mode
// reads the fill copy or substitutes on the fly.
ReqDesc make_desc(const Matrix &m, int32_t n, const int32_t *offsets, const int32_t *cols,
                  uint32_t flags, int32_t *matched, int32_t *negative, uint64_t *mmask,
                  uint64_t *nmask, int32_t staging);
// At least `bytes` of device scratch private to stream `s` (grown on demand;
// a grown buffer replaces the old one after the stream has drained).
void *stream_scratch(ebic_ctx *ctx, hipStream_t s, size_t bytes);
// The upload's two pinned host buffers, at least `bytes` each (under mu).
void upload_pinned(ebic_ctx *ctx, size_t bytes);
// Copy rows [r0, r0 + nr) of a host matrix (row-major with row stride
// ld_src, or column-major with column stride ld_src) into dst, packed
// (row-major: nr x cols; column-major: cols x nr), with a few threads.
void pack_rows(const float *src, int64_t ld_src, bool col_major, int64_t r0, int64_t nr, int32_t cols,
               float *dst);
// Launch one evaluation with the context's diagnostics applied.
hipError_t ctx_launch_eval(ebic_ctx *ctx, const ReqDesc &d, const LaunchCfg &cfg, hipStream_t s);

// ebic_tune.cpp
TuneKey tune_key(int64_t rows, int32_t cols, int32_t n, int64_t nnz);
LaunchCfg tuned_cfg(ebic_ctx *ctx, int64_t rows, int32_t cols, int32_t n, int64_t nnz);
LaunchCfg tuned_batch_cfg(ebic_ctx *ctx, int64_t total_ind, int64_t mean_rows, int32_t max_cols,
                          int64_t nnz);
LaunchCfg default_batch_cfg(int32_t max_cols);
LaunchCfg default_batch_codes_cfg(int32_t max_cols);  // (the shape without the pair bitmaps)
LaunchCfg default_cfg(int64_t rows, int32_t cols, int32_t n);
LaunchCfg default_codes_cfg(int64_t rows, int32_t cols, int32_t n);  // (the shape without the pair bitmaps)
void load_tune_cache(ebic_ctx *ctx, const std::string &path);

// ebic_batch.cpp
void destroy_batch_state(ebic_ctx *ctx);

}  // namespace ebic

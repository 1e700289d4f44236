// ebic_internal.h -- declarations shared by the runtime (ebic_runtime.cpp)
// and the kernels (ebic_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebic {

// How the column tile of a work item reaches the predicate.
enum Staging : int32_t {
    STAGE_LDS = 0,     // rows x all columns staged into LDS, shared by the block
    STAGE_DIRECT = 1,  // read straight from the column-major matrix (L1/L2)
};

// One launch shape of the evaluation kernels.
struct LaunchCfg {
    int32_t L = 0;        // 64-row sub-tiles evaluated together per wave (1, 2, 4)
    int32_t W = 0;        // waves per block (1..16)
    int32_t P = 0;        // individuals per group (max individuals sharing a block)
    int32_t staging = STAGE_LDS;
    int32_t blocks = 0;   // grid size (x); 0 = derive from occupancy
};

// A resident matrix as the kernels see it.
struct DevMatrix {
    const float *X = nullptr;      // column-major, leading dimension ld
    const float *Xfill = nullptr;  // fill-substituted copy, or null
    int64_t ld = 0;                // multiple of 64
    int64_t rows = 0;
    int32_t cols = 0;
    float fill = 0.f;
};

// Arguments of one population evaluation.
struct EvalArgs {
    DevMatrix m;
    const int32_t *offsets = nullptr;
    const int32_t *cols = nullptr;
    int32_t n = 0;
    uint32_t flags = 0;
    int32_t *matched = nullptr;
    int32_t *negative = nullptr;
    uint64_t *mmask = nullptr;
    uint64_t *nmask = nullptr;
    // Diagnostics: when not null, every wave adds the number of (column,
    // 64-row sub-tile) predicate steps it executed (selects a counting
    // variant of the kernel).
    unsigned long long *step_counter = nullptr;
};

// Bytes of dynamic LDS a launch shape needs.
size_t eval_lds_bytes(const LaunchCfg &cfg, int32_t cols);

// Blocks per CU the evaluation kernel reaches with this shape (0 = cannot run).
int eval_occupancy(const LaunchCfg &cfg, int32_t cols, uint32_t flags);

// Enqueue: validation/zeroing of the outputs, then the evaluation kernel.
// If ev0/ev1 are not null they are recorded on `s` right before and right
// after the evaluation kernel.
hipError_t launch_eval(const EvalArgs &a, const LaunchCfg &cfg, hipStream_t s,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Enqueue the layout kernel: src (device, row-major with row stride ld_src,
// or column-major with column stride ld_src) -> dst column-major with
// leading dimension ld; rows [r0, r0 + nr) of the matrix; cells equal to the
// sentinel become NaN; if dst_fill is not null it receives the same values
// with every missing cell replaced by `fill`.
hipError_t launch_layout(const float *src, int64_t ld_src, bool src_col_major, int64_t nr,
                         int32_t cols, int64_t r0, float *dst, int64_t ld, float sentinel,
                         float *dst_fill, float fill, hipStream_t s);

// Zero rows [rows, ld) of every column of a column-major matrix.
hipError_t launch_zero_pad(float *dst, int64_t rows, int64_t ld, int32_t cols, hipStream_t s);

}  // namespace ebic

// ebic_layout.hip -- upload kernels: the resident matrix layout.
//
// The matrix is kept column-major (one column of 64 consecutive rows is one
// coalesced 256-byte segment for a wave) with a leading dimension padded to
// a multiple of 64 rows; padding rows hold 0. Missing cells are stored as
// NaN: the paper lets the user mark missing values with a predefined value
// (Methods, "Handling missing values"), so cells equal to that sentinel are
// converted here. An optional second copy holds the fill value in place of
// every missing cell, for the mode in which missing values take part in the
// comparison.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebic_internal.h"

namespace ebic {

namespace {

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

// ---------------------------------------------------------------------------
// Rank codes: for every cell, the number of cells of its row that are
// smaller (IEEE <, so NaN is never smaller and -0 is not smaller than +0),
// as an FP16 integer; a missing cell gets NaN. A block stages 64 rows of all
// columns in LDS; thread (lane, wave) counts, for its row, the columns wave,
// wave + 4, ... Padding rows get code 0.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_codes(const float *__restrict__ X, int64_t rows, int64_t ld, int32_t cols, uint16_t *__restrict__ C)
{
    extern __shared__ float t[];  // [cols][64]
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int32_t c = wave; c < cols; c += 4) t[c * 64 + lane] = X[(int64_t)c * ld + r0 + lane];
    __syncthreads();
    const bool live = r0 + lane < rows;
    for (int32_t c = wave; c < cols; c += 4) {
        const float v = t[c * 64 + lane];
        int32_t n = 0;
        for (int32_t j = 0; j < cols; ++j) n += t[j * 64 + lane] < v ? 1 : 0;
        uint16_t code = __half_as_ushort(__int2half_rn(n));  // exact: n < 2048
        if (v != v) code = kCodeNaN;
        C[(int64_t)c * ld + r0 + lane] = live ? code : (uint16_t)0;
    }
}

// ---------------------------------------------------------------------------
// Byte or 16-bit rank codes: as above, of the fill-substituted values, in
// the interleaved order of the SWAR evaluation. Bytes: within each 256-row
// group the word of lane l holds rows l, 64 + l, 128 + l, 192 + l; 16 bits:
// within each 128-row group it holds rows l and 64 + l. Rows past the
// matrix get 0. Also flags any missing cell, and each 512-row group with a
// row that holds two equal values.
// ---------------------------------------------------------------------------
template <typename C>
__global__ void __launch_bounds__(256)
k_swar_codes(const float *__restrict__ X, int64_t rows, int64_t ld, int32_t cols, float fill,
             C *__restrict__ out, int64_t ld_out, int32_t *__restrict__ has_nan, int32_t *__restrict__ ties)
{
    extern __shared__ float t[];  // [cols][64]
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = r0 + lane;
    const bool live = r < rows;
    bool missing = false;
    for (int32_t c = wave; c < cols; c += 4) {
        float v = live ? X[(int64_t)c * ld + r] : 0.f;
        if (v != v) {
            missing = true;
            v = fill;
        }
        t[c * 64 + lane] = v;
    }
    if (missing) *has_nan = 1;
    __syncthreads();
    // Position of row r (in elements of C) inside its interleaved group.
    const int64_t pos = sizeof(C) == 1 ? (r & ~(int64_t)255) + 4 * (r & 63) + ((r >> 6) & 3)
                                       : (r & ~(int64_t)127) + 2 * (r & 63) + ((r >> 6) & 1);
    bool tie = false;
    for (int32_t c = wave; c < cols; c += 4) {
        const float v = t[c * 64 + lane];
        int32_t n = 0, e = 0;
        for (int32_t j = 0; j < cols; ++j) {
            const float u = t[j * 64 + lane];
            n += u < v ? 1 : 0;
            e += u == v ? 1 : 0;
        }
        tie |= e > 1;  // another cell of the row has the same value (and code)
        out[(int64_t)c * ld_out + pos] = live ? (C)n : (C)0;
    }
    if (live && tie) ties[r >> 9] = 1;
}

// 10-bit rank codes: the same counts, three rows per 32-bit word. Block b
// holds rows [64 b, 64 b + 64), which are field b mod 3 of 192-row group
// b / 3: each code is OR-ed into its word (the three blocks of a group
// write disjoint fields of the same words). Flags a missing cell, and each
// 192-row group with a row that holds two equal values.
__global__ void __launch_bounds__(256)
k_t10_codes(const float *__restrict__ X, int64_t rows, int64_t ld, int32_t cols, float fill,
            uint32_t *__restrict__ out, int64_t ld_words, int32_t *__restrict__ has_nan,
            int32_t *__restrict__ ties)
{
    extern __shared__ float t[];  // [cols][64]
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = r0 + lane;
    const bool live = r < rows;
    bool missing = false;
    for (int32_t c = wave; c < cols; c += 4) {
        float v = live ? X[(int64_t)c * ld + r] : 0.f;
        if (v != v) {
            missing = true;
            v = fill;
        }
        t[c * 64 + lane] = v;
    }
    if (missing) *has_nan = 1;
    __syncthreads();
    const int64_t group = blockIdx.x / 3;
    const int field = blockIdx.x % 3;
    bool tie = false;
    for (int32_t c = wave; c < cols; c += 4) {
        const float v = t[c * 64 + lane];
        uint32_t n = 0, e = 0;
        for (int32_t j = 0; j < cols; ++j) {
            const float u = t[j * 64 + lane];
            n += u < v ? 1u : 0u;
            e += u == v ? 1u : 0u;
        }
        tie |= e > 1;
        if (live && n) atomicOr(out + (int64_t)c * ld_words + group * 64 + lane, n << (10 * field));
    }
    if (live && tie) ties[group] = 1;
}

__global__ void k_zero_pad(float *__restrict__ dst, int64_t rows, int64_t ld, int32_t cols)
{
    const int64_t pad = ld - rows;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= pad * cols) return;
    const int64_t c = idx / pad, r = rows + idx % pad;
    dst[c * ld + r] = 0.f;
}

}  // namespace

hipError_t launch_codes(const float *X, int64_t rows, int64_t ld, int32_t cols, uint16_t *C,
                        hipStream_t s)
{
    if (cols > kMaxCodeCols) return hipErrorInvalidValue;
    const size_t lds = (size_t)cols * 64 * sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_codes),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    clear_last_error();
    hipLaunchKernelGGL(k_codes, dim3((unsigned)(ld / 64)), dim3(256), lds, s, X, rows, ld, cols, C);
    return hipGetLastError();
}

hipError_t launch_byte_codes(const float *X, int64_t rows, int64_t ld, int32_t cols, float fill,
                             uint8_t *B, int64_t ldb, int32_t *has_nan, int32_t *ties, hipStream_t s)
{
    if (cols > kMaxByteCols || ldb % 512 != 0 || ldb < rows) return hipErrorInvalidValue;
    const size_t lds = (size_t)cols * 64 * sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_swar_codes<uint8_t>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    clear_last_error();
    hipLaunchKernelGGL(k_swar_codes<uint8_t>, dim3((unsigned)(ldb / 64)), dim3(256), lds, s, X, rows, ld,
                       cols, fill, B, ldb, has_nan, ties);
    return hipGetLastError();
}

hipError_t launch_half_codes(const float *X, int64_t rows, int64_t ld, int32_t cols, float fill,
                             uint8_t *Hc, int64_t ldh, int32_t *has_nan, int32_t *ties, hipStream_t s)
{
    if (cols > kMaxCodeCols || ldh % 512 != 0 || ldh / 2 < rows) return hipErrorInvalidValue;
    const size_t lds = (size_t)cols * 64 * sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_swar_codes<uint16_t>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    clear_last_error();
    hipLaunchKernelGGL(k_swar_codes<uint16_t>, dim3((unsigned)(ldh / 2 / 64)), dim3(256), lds, s, X, rows,
                       ld, cols, fill, reinterpret_cast<uint16_t *>(Hc), ldh / 2, has_nan, ties);
    return hipGetLastError();
}

hipError_t launch_t10_codes(const float *X, int64_t rows, int64_t ld, int32_t cols, float fill,
                            uint8_t *T10, int64_t ld10, int32_t *has_nan, int32_t *ties, hipStream_t s)
{
    const int64_t groups = (rows + kT10Rows - 1) / kT10Rows;
    if (cols > kMaxT10Cols || ld10 < groups * 256 || ld10 % 256 != 0 || ld / 64 < (rows + 63) / 64)
        return hipErrorInvalidValue;
    const size_t lds = (size_t)cols * 64 * sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_t10_codes),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // one block per 64 rows up to the last group's end; X is read only for
    // rows below `rows`
    clear_last_error();
    hipLaunchKernelGGL(k_t10_codes, dim3((unsigned)(groups * 3)), dim3(256), lds, s, X, rows, ld, cols, fill,
                       reinterpret_cast<uint32_t *>(T10), ld10 / 4, has_nan, ties);
    return hipGetLastError();
}

hipError_t launch_layout(const float *src, int64_t ld_src, bool src_col_major, int64_t nr,
                         int32_t cols, int64_t r0, float *dst, int64_t ld, float sentinel,
                         float *dst_fill, float fill, hipStream_t s)
{
    if (nr <= 0) return hipSuccess;
    dim3 grid((unsigned)((nr + 63) / 64), (unsigned)((cols + 63) / 64));
    clear_last_error();
    hipLaunchKernelGGL(k_layout, grid, dim3(256), 0, s, src, ld_src, (int32_t)src_col_major, nr,
                       cols, r0, dst, ld, sentinel, dst_fill, fill);
    return hipGetLastError();
}

hipError_t launch_zero_pad(float *dst, int64_t rows, int64_t ld, int32_t cols, hipStream_t s)
{
    const int64_t total = (ld - rows) * cols;
    if (total <= 0) return hipSuccess;
    const int threads = 256;
    clear_last_error();
    hipLaunchKernelGGL(k_zero_pad, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads),
                       0, s, dst, rows, ld, cols);
    return hipGetLastError();
}

}  // namespace ebic

// ebic_internal.h -- declarations shared by the runtime (ebic_runtime.cpp,
// ebic_batch.cpp, ebic_tune.cpp) and the kernels (ebic_eval.hip,
// ebic_layout.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebic {

constexpr int kWave = 64;  // gfx950 wavefront
constexpr int kWin = 8;    // leading columns of an individual kept in its header

// How the column tile of a work item reaches the predicate.
enum Staging : int32_t {
    STAGE_LDS = 0,     // rows x all columns staged into LDS, shared by the block
    STAGE_DIRECT = 1,  // read straight from the column-major matrix (L1/L2)
    STAGE_CODES = 2,   // the matrix's 16-bit rank codes staged into LDS (half the bytes)
    STAGE_BYTES = 3,   // 8-bit rank codes, four rows per 32-bit lane word (4 or 8 sub-tiles)
    STAGE_HALVES = 4,  // 16-bit rank codes, two rows per 32-bit lane word (4 sub-tiles)
    STAGE_T10 = 5,     // 10-bit rank codes, three rows per 32-bit lane word (3 sub-tiles)
    STAGE_PAIRS = 6,   // pairwise order bitmaps, 32 rows per lane word, nothing staged
};

// Rank codes are kept for matrices of at most this many columns: a cell's
// code is the number of cells of its row that are smaller, stored as an
// FP16 integer (exact up to 2048), NaN for a missing cell. Codes compare
// exactly as the values do (a >= b iff code(a) >= code(b)), so the
// predicate on codes gives the same rows.
constexpr int32_t kMaxCodeCols = 384;
constexpr uint16_t kCodeNaN = 0x7E00;

// Byte rank codes, for matrices of at most 128 columns: the same count of
// smaller cells, of the fill-substituted values (so there is no missing
// code), as one byte. Within each group of 256 rows the bytes are ordered
// so that the 32-bit word of lane l holds rows l, 64 + l, 128 + l and
// 192 + l (bytes 0..3): one word per lane covers four 64-row sub-tiles, and
// byte b of all lanes is sub-tile b. A column occupies ldb bytes, ldb =
// rows rounded up to a multiple of 256; padding rows hold 0. Exclude mode
// may use them only when the matrix has no missing cell.
constexpr int32_t kMaxByteCols = 128;

// 16-bit rank codes, for matrices of at most kMaxCodeCols columns: the same
// codes of the fill-substituted values in 16 bits. Within each group of 128
// rows the 32-bit word of lane l holds rows l and 64 + l (low and high
// half). A column occupies ldh bytes (rows rounded up to a multiple of 256,
// two bytes each); exclude mode may use them only without missing cells.

// 10-bit rank codes, for matrices of 129 to 512 columns: the same codes of
// the fill-substituted values (0..511), three per 32-bit word in fields of
// ten bits (bits 0-8, 10-18 and 20-28 hold the codes; bits 9, 19 and 29 are
// the fields' top bits, 30-31 stay zero). Within each 192-row group the
// word of lane l holds rows l, 64 + l and 128 + l (fields 0, 1, 2). A
// column occupies ld10 bytes (256 per 192-row group); exclude mode may use
// them only without missing cells. One tie flag per 192-row group.
constexpr int32_t kMaxT10Cols = 512;
constexpr int32_t kT10Rows = 192;  // rows per lane-word group

// Request flags as the kernels see them (the low two bits are the ABI's
// EBIC_NAN_INCLUDE and EBIC_NEG_TRENDS).
constexpr uint32_t kFlagInclude = 1u;
constexpr uint32_t kFlagNeg = 2u;
constexpr uint32_t kFlagDirect = 1u << 8;  // this request reads the matrix directly
constexpr uint32_t kFlagSubst = 1u << 9;   // direct reads replace NaN by the fill value
constexpr uint32_t kFlagCodes = 1u << 10;  // this request stages the rank codes
constexpr uint32_t kFlagBytes = 1u << 11;  // this request stages the byte rank codes
constexpr uint32_t kFlagHalves = 1u << 12; // this request stages the 16-bit rank codes
constexpr uint32_t kFlagT10 = 1u << 13;    // this request stages the 10-bit rank codes
constexpr uint32_t kFlagPairs = 1u << 14;  // this request reads the pairwise order bitmaps

// One launch shape of the evaluation kernels.
struct LaunchCfg {
    int32_t L = 0;        // 64-row sub-tiles evaluated together per wave (1, 2, 4; codes: 2, 4; bytes: 4)
    int32_t W = 0;        // waves per block (1..16)
    int32_t P = 0;        // individuals per group (max individuals sharing a block)
    int32_t staging = STAGE_LDS;
    int32_t blocks = 0;   // plain: tile ranges per group; batch: persistent grid; 0 = derive
    bool cnt16 = false;   // plain: counts as 16-bit halves (16-bit codes; set by the planner)
};

// A resident matrix as the kernels see it.
struct DevMatrix {
    const float *X = nullptr;      // column-major, leading dimension ld, missing = NaN
    const float *Xfill = nullptr;  // fill-substituted copy, or null
    const uint16_t *C = nullptr;   // rank codes of X (same layout), or null
    const uint16_t *Cfill = nullptr;  // rank codes of Xfill, or null
    const uint8_t *B = nullptr;    // byte rank codes of the fill-substituted values, or null
    const int32_t *T = nullptr;    // per 512-row group of B: 1 if a row has two equal values
    const uint8_t *Hc = nullptr;   // 16-bit rank codes (interleaved, as bytes), or null
    const int32_t *Th = nullptr;   // their tie flags per 512 rows
    bool h_exclude = false;        // Hc also serves exclude mode (no missing cell)
    int64_t ldh = 0;               // bytes per column of Hc (multiple of 512)
    const uint8_t *T10 = nullptr;  // 10-bit rank codes (three rows per word), or null
    const int32_t *Tt = nullptr;   // their tie flags per 192-row group
    bool t_exclude = false;        // T10 also serves exclude mode (no missing cell)
    int64_t ld10 = 0;              // bytes per column of T10 (256 per 192 rows)
    bool b_exclude = false;        // B also serves exclude mode (no missing cell)
    int64_t ldb = 0;               // bytes per column of B (multiple of 256)
    const uint32_t *Gx = nullptr;  // pairwise order bitmaps of X (exclude mode), or null
    const uint32_t *Gf = nullptr;  // of the fill-substituted values (include mode), or null
    int64_t w32 = 0;               // 32-bit words per pair (whole 2048-row chunks)
    int64_t ld = 0;                // multiple of 64
    int64_t rows = 0;
    int32_t cols = 0;
    float fill = 0.f;
};

// One population evaluation as the kernels read it.
struct ReqDesc {
    const float *X;            // the matrix to read (the fill copy when it serves include mode)
    const uint16_t *C;         // the rank codes to stage (kFlagCodes), or null
    const uint8_t *B;          // the byte, 16-bit or 10-bit rank codes to stage (kFlagBytes, kFlagHalves,
                               // kFlagT10), or the pairwise order bitmaps (kFlagPairs; ldb = words per pair)
    const int32_t *T;          // their per-512-row tie flags
    int64_t ldb;               // bytes per column of B
    int64_t ld;
    int64_t rows;
    int32_t cols;
    float fill;
    uint32_t flags;            // kFlag*
    int32_t n;                 // individuals
    const int32_t *offsets;    // CSR, n + 1 entries
    const int32_t *colidx;
    int32_t *matched;
    int32_t *negative;         // may be null
    uint64_t *mmask;           // may be null
    uint64_t *nmask;           // may be null
    int64_t head_base;         // first row of this request in the header table
};

// Per-individual header written by the prep kernel (64 bytes, one scalar
// load): k = length (0 for an invalid individual), the CSR start of its
// columns, and its first kWin columns (clamped to the last one).
struct IndHead {
    int32_t k;
    int32_t begin;
    int32_t pad[6];
    int32_t win[kWin];
};
static_assert(sizeof(IndHead) == 64, "IndHead is one 64-byte scalar load");

// A work item of the batched kernel: individuals [i0, i0 + np) of request
// `req`, on 64-row tiles [t0, t1).
struct Item {
    int32_t req;
    int32_t i0;
    int32_t np;
    int32_t t0;
    int32_t t1;
    int32_t pad[3];
};
static_assert(sizeof(Item) == 32, "Item is 32 bytes");

// Device-side header of a batch: counts and the dynamic work counter.
struct BatchHeader {
    int32_t n_req;
    int32_t n_items;
    int64_t total_ind;     // individuals over all requests
    uint32_t counter;      // next item to take (zeroed by the prep kernel)
    uint32_t pad[3];
};

// Bytes of dynamic LDS one work item needs: the staged tile (if staged) and
// the per-individual counts of a group of P.
size_t tile_lds_bytes(int32_t L, int32_t cols, int32_t staging);
size_t count_lds_bytes(int32_t P);
// All dynamic LDS of one plain-evaluation item (tile and counts; cnt16:
// both counts of an individual in one 32-bit word).
size_t item_lds_bytes(int32_t L, int32_t cols, int32_t staging, int32_t P, bool cnt16 = false);

// Blocks per CU the plain evaluation kernel reaches with this shape (0 = cannot run).
int eval_occupancy(const LaunchCfg &cfg, int32_t cols, uint32_t flags);
// Stagings a batched launch handles (the kernel instance is picked by the set
// its requests use: one kind of SWAR codes alone, or all).
constexpr int32_t kBatchSetBytes = 1;
constexpr int32_t kBatchSetHalves = 2;
constexpr int32_t kBatchSetCodes = 4;
constexpr int32_t kBatchSetValues = 8;  // the FP32 tile or direct reads
constexpr int32_t kBatchSetT10 = 16;
constexpr int32_t kBatchSetAll = 31;
// The sub-tiles per chunk of a request that stages `staging` in a batch
// whose FP32/FP16 stagings take L: SWAR codes fix their own.
inline int32_t batch_tiles(int32_t staging, int32_t L)
{
    return staging == STAGE_BYTES ? 4 : staging == STAGE_T10 ? 3 : staging == STAGE_HALVES ? 2 : L;
}
int batch_occupancy(int32_t L, int32_t set, int32_t W, size_t lds_bytes);

// Plain evaluation: prep (validation, output initialisation, headers) then
// the evaluation kernel over G groups x cfg.blocks tile ranges. ev0/ev1, if
// not null, are recorded right before and after the evaluation kernel.
hipError_t launch_eval(const ReqDesc &d, IndHead *heads, const LaunchCfg &cfg,
                       unsigned long long *step_counter, hipStream_t s,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// The no-allocation evaluation's header buffer: a fixed device array of
// kNoAllocMaxInd headers per device. noalloc_scratch_init (called with
// `device` current, once per device, at context creation) looks up its
// device address; noalloc_scratch returns it (null before the init).
constexpr int32_t kNoAllocMaxInd = 65536;
hipError_t noalloc_scratch_init(int device);
IndHead *noalloc_scratch(int device);

// Batched evaluation over a device-resident batch arena:
//   hdr (BatchHeader) | descs (ReqDesc[n_req]) | first (int64[n_req + 1],
//   prefix sums of individuals) | items (Item[n_items])
// prep_blocks x 256 threads validate every individual of every request;
// then `grid` persistent blocks of W waves take items from the counter.
hipError_t launch_batch(BatchHeader *hdr, const ReqDesc *descs, const int64_t *first,
                        const Item *items, IndHead *heads, int32_t L, int32_t set, int32_t W, int32_t P,
                        size_t tile_bytes, int32_t grid, int32_t prep_blocks,
                        unsigned long long *step_counter, hipStream_t s,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Layout kernel: src (device, row-major with row stride ld_src, or
// column-major with column stride ld_src), rows [r0, r0 + nr) of the matrix
// -> dst column-major with leading dimension ld; cells equal to the sentinel
// become NaN; if dst_fill is not null it receives the same values with every
// missing cell replaced by `fill`.
hipError_t launch_layout(const float *src, int64_t ld_src, bool src_col_major, int64_t nr,
                         int32_t cols, int64_t r0, float *dst, int64_t ld, float sentinel,
                         float *dst_fill, float fill, hipStream_t s);

// Rank codes of rows [0, rows) of a column-major matrix (cols <= kMaxCodeCols),
// written column-major with the same leading dimension; padding rows get 0.
hipError_t launch_codes(const float *X, int64_t rows, int64_t ld, int32_t cols, uint16_t *C,
                        hipStream_t s);

// Byte rank codes of rows [0, rows) of a column-major matrix (cols <=
// kMaxByteCols), with missing cells replaced by `fill`, into B (ldb bytes
// per column, ldb a multiple of 512, the interleaved order above; padding
// rows get 0). *has_nan (device int, zeroed by the caller) is set to 1 if
// any cell is missing; ties[g] (ldb / 512 device ints, zeroed by the
// caller) is set to 1 if some row of rows [512 g, 512 g + 512) holds two
// equal values.
hipError_t launch_byte_codes(const float *X, int64_t rows, int64_t ld, int32_t cols, float fill,
                             uint8_t *B, int64_t ldb, int32_t *has_nan, int32_t *ties, hipStream_t s);

// The same for 16-bit codes (cols <= kMaxCodeCols) into Hc, ldh bytes per
// column (a multiple of 512), in their interleaved order.
hipError_t launch_half_codes(const float *X, int64_t rows, int64_t ld, int32_t cols, float fill,
                             uint8_t *Hc, int64_t ldh, int32_t *has_nan, int32_t *ties, hipStream_t s);

// The same for 10-bit codes (cols <= kMaxT10Cols) into T10, ld10 bytes per
// column (256 per 192-row group; T10 zeroed by the caller, the fields are
// OR-ed in), and one tie flag per 192-row group.
// Clears the calling thread's last HIP error before a launch, so that the
// hipGetLastError() after it reports that launch's own error (not one an
// earlier call left, such as an ignored error of a release path).
inline void clear_last_error() { (void)hipGetLastError(); }

// Pairwise order bitmaps (ebic_pairs.hip): words per pair for `rows`, the
// build of every pair's words from a column-major matrix (subst: NaN takes
// `fill` first) with each 2,048-row chunk's list of tied pairs and NaN flag
// in T (pair_tie_bytes, zeroed by the caller), the prep kernel writing the
// pairs headers, the evaluation kernel for request flags (ReqDesc: B = the
// words, T = the tie lists), and its grid.
constexpr int32_t kMaxPairCols = 1024;
constexpr int64_t kMaxPairRows = 65535ll * 8 * 2048;  // (the plain launch's grid: chunks / 8 in y)
constexpr int32_t kDefaultPairCols = 512;  // widths planned on the bitmaps unless a shape says otherwise
constexpr int64_t kMaxPairBytes = 32ll << 30;
int64_t pair_words(int64_t rows);
int64_t pair_tie_bytes(int64_t rows);
hipError_t launch_pair_bits(const float *X, int64_t rows, int64_t ld, int32_t cols, bool subst, float fill,
                            uint32_t *G, int64_t w32, uint32_t *T, hipStream_t s);
hipError_t launch_prep_pairs(const ReqDesc &d, IndHead *heads, hipStream_t s);
const void *pairs_kernel(uint32_t flags, bool count, int32_t P, int32_t W);
dim3 pairs_grid(int64_t rows, int32_t n, int32_t P);

// The pair items of a batch: eight lists, one per XCD slice (a slice: the
// chunks c with c mod 8 = x), each walking its chunks in order segment by
// segment; a segment is the requests reading one set of bitmaps, listed in
// the entries e0 .. e0 + n_req - 1 of seg_req (request index) and seg_gstart
// (the request's first group within the segment, groups of P individuals).
struct PairQueues {
    int32_t total[8];  // items per list
    int32_t n_seg;
    int32_t P;         // individuals per group (at most 64 per wave)
    int32_t pad[6];
};
struct PairSeg {
    int32_t e0, n_req;
    int32_t groups;    // groups over the segment's requests
    int32_t n_chunks;  // 2,048-row chunks of its matrix
    int32_t base[8];   // the segment's first item in each list
};
hipError_t launch_pairs_batch(const PairQueues *pq, const ReqDesc *descs, const PairSeg *segs,
                              const int32_t *seg_req, const int32_t *seg_gstart, const IndHead *heads, int32_t W,
                              int32_t grid, unsigned long long *step_counter, hipStream_t s);
int pairs_batch_occupancy(int32_t W);  // blocks per CU of the batched pairs kernel
hipError_t launch_t10_codes(const float *X, int64_t rows, int64_t ld, int32_t cols, float fill,
                            uint8_t *T10, int64_t ld10, int32_t *has_nan, int32_t *ties, hipStream_t s);

// Zero rows [rows, ld) of every column of a column-major matrix.
hipError_t launch_zero_pad(float *dst, int64_t rows, int64_t ld, int32_t cols, hipStream_t s);

}  // namespace ebic

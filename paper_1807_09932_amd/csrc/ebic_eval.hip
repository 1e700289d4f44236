// ebic_eval.hip -- gfx950 kernels of the EBIC fitness evaluation.
//
// The evaluation counts, for every individual (an ordered column list
// c_0..c_{k-1}), the rows whose values follow the >= chain along that order,
// and optionally the reversed (<=) chain (EBIC paper, Methods, "Handling
// missing values"; rows up to 2^31-1 per GPU, Methods, "Support for Big
// Data"). All outputs are integers decided by exact FP32 compares.
//
// Work decomposition. A work item is (a group of up to P individuals of one
// population, a contiguous range of 64-row tiles of its matrix, starting on
// a multiple of L tiles). The block that owns an item walks the range L
// tiles at a time: it stages those L*64 rows of every column into LDS
// (column-major, so lane l of a wave reads bank l; rows outside the item or
// the matrix hold NaN), then each wave takes every W-th individual of the
// group and evaluates it on the L sub-tiles: lane l holds row l of each
// sub-tile. After the first pair of columns each row follows one oriented
// chain (falling rows are sign-flipped), so every further column is one XOR
// and one compare per sub-tile, reduced across the wave into a 64-bit alive
// mask in scalar registers. With L = 2 or 4 the sub-tiles run interleaved in
// one instruction stream (independent compares hide each other's latency);
// the individual stops as soon as no row of its L sub-tiles can still match
// (a wave-uniform early exit). Counts are popcounts of the masks,
// accumulated per block in LDS and added to global memory once per item with
// integer atomics (order-independent, so results are deterministic).
//
// The plain kernel (one population) launches one block per item on a 2-D
// grid. The batched kernel (many populations, many matrices) is persistent:
// its blocks take items from a device-side counter until none are left.
//
// Before either, a prep kernel validates every individual, initialises its
// outputs (0, or -1 for an invalid individual) and writes its 64-byte header
// (length, CSR start, first kWin columns clamped to the last one), which the
// evaluation reads with one scalar load per individual.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <type_traits>

#include "ebic_internal.h"
#include "ebic_prep.h"

namespace ebic {

namespace {

__host__ __device__ inline size_t tile_bytes_of(int32_t L, int32_t cols, int32_t staging)
{
    if (staging == STAGE_DIRECT || staging == STAGE_PAIRS) return 0;
    if (staging == STAGE_BYTES) return (size_t)cols * L * kWave;  // one byte per row
    if (staging == STAGE_HALVES) return (size_t)cols * L * kWave * 2;
    if (staging == STAGE_T10) return (size_t)cols * 256 * (L >= 6 ? 2 : 1);  // one or two lane words
    return (size_t)L * kWave * cols * (staging == STAGE_CODES ? sizeof(uint16_t) : sizeof(float));
}

// Per-individual [matched, negative] counts of a group of P: two 32-bit
// words each, or (cnt16) one word holding both as 16-bit halves.
__host__ __device__ inline size_t count_bytes_of(int32_t P, bool cnt16 = false)
{
    return (size_t)((P + 1) & ~1) * (cnt16 ? 1 : 2) * sizeof(int32_t);
}

// ---------------------------------------------------------------------------
// Prep: validation, output initialisation and the per-individual header.
// ---------------------------------------------------------------------------
// One wave per individual (the scan of its columns, with the leading
// repeats of the first column dropped, in ebic_prep.h): lane 0 initialises
// the outputs, and lanes 0..15 write the 64-byte header word by word.
__device__ __forceinline__ void prep_wave(const ReqDesc &d, int32_t i, IndHead *__restrict__ heads, int lane)
{
    const PrepScan sc = prep_scan(d, i, lane);
    if (lane == 0) {
        d.matched[i] = sc.ok ? 0 : kInvalid;
        if (d.negative) d.negative[i] = sc.ok ? 0 : kInvalid;
    }
    if (lane < 16) {
        // words: k, begin, 6 x 0, the window
        const int32_t v = lane == 0 ? sc.k : lane == 1 ? sc.bb : (lane >= 8 && sc.ok) ? sc.win : 0;
        reinterpret_cast<int32_t *>(heads + d.head_base + i)[lane] = v;
    }
}

__global__ void __launch_bounds__(256) k_prep(ReqDesc d, IndHead *__restrict__ heads)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int32_t i = blockIdx.x * (blockDim.x / kWave) + wave;
    if (i < d.n) prep_wave(d, i, heads, threadIdx.x & (kWave - 1));
}

__global__ void __launch_bounds__(256) k_prep_batch(BatchHeader *hdr, const ReqDesc *__restrict__ descs,
                                                    const int64_t *__restrict__ first, IndHead *__restrict__ heads)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) hdr->counter = 0;
    const int64_t total = hdr->total_ind;
    const int32_t nreq = hdr->n_req;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t g = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave; g < total; g += stride) {
        int32_t lo = 0, hi = nreq - 1;  // the last request with first[q] <= g
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (first[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        if (descs[lo].flags & kFlagPairs)
            prep_pairs_wave(descs[lo], (int32_t)(g - first[lo]), heads, threadIdx.x & (kWave - 1));
        else
            prep_wave(descs[lo], (int32_t)(g - first[lo]), heads, threadIdx.x & (kWave - 1));
    }
}

// ---------------------------------------------------------------------------
// The predicate.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// The predicate on LDS-staged tiles, as one oriented chain per row.
//
// After the first pair (c_0, c_1) every row that can still match follows
// one direction: rows with v_1 > v_0 can only be on the >= chain, rows with
// v_1 < v_0 only on the <= chain. Flipping the sign bit of every value of a
// falling row (an exact negation, also for +-0, +-inf and NaN) turns its
// <= chain into a >= chain, so from the second pair on every row runs the
// same test, (v_j ^ flip) >= (v_{j-1} ^ flip), and the wave carries one
// alive mask: the execution mask. Each column step is an XOR and a compare
// (VALU) and one AND into the execution mask (SALU); the chain stops for
// the wave as soon as no row is left (s_cbranch_execz). Rows tied on the
// first pair (v_1 == v_0) follow the >= chain here and get a second chain
// for the <= direction. NaN compares false, so a missing value anywhere
// along the chain removes the row (exclude mode); in include mode the tile
// holds no NaN.
// ---------------------------------------------------------------------------
constexpr uint32_t kSign = 0x80000000u;

typedef __attribute__((address_space(3))) const unsigned char lds_uchar;

// Byte offset of an LDS pointer in the LDS address space.
__device__ __forceinline__ uint32_t lds_addr(const void *p)
{
    return (uint32_t)(uintptr_t)(lds_uchar *)p;
}

__device__ __forceinline__ float flipped(float v, uint32_t flip)
{
    return __uint_as_float(__float_as_uint(v) ^ flip);
}

// The window's column steps 2..min(last, 7), as assembly text shared by the
// sequences below: three pairs of columns; for each column an XOR (omitted
// when every row runs the >= chain), a compare into VCC and an AND of VCC
// into EXEC; after each pair the chain ends if no row is left
// (s_cbranch_execz) or if the individual has no more columns. The loads of
// the next pair are issued before the current pair is compared, so LDS
// latency overlaps the compares. The sequence starts with lgkmcnt(0) (no
// scalar load of the surrounding code in flight, so LDS loads complete in
// issue order and lgkmcnt(2) names the older pair) and ends with it (no
// load left in flight when control returns). `prev` holds the (flipped)
// value of column 1; the first pair's loads are issued by the caller's text.
#define EBIC_XOR(r) "v_xor_b32 %[" r "], %[" r "], %[flip]\n\t"
#define EBIC_CMP2(ra, rb, rp, XORA, XORB)                                      \
    XORA                                                                       \
    "v_cmp_ge_f32 vcc, %[" ra "], %[" rp "]\n\t"                               \
    XORB                                                                       \
    "s_and_b64 exec, exec, vcc\n\t"                                            \
    "v_cmp_ge_f32 vcc, %[" rb "], %[" ra "]\n\t"                               \
    "s_and_b64 exec, exec, vcc\n\t"
#define EBIC_LOAD2(ra, rb, aa, ab)                                             \
    "ds_read_b32 %[" ra "], %[" aa "] offset:%[off]\n\t"                       \
    "ds_read_b32 %[" rb "], %[" ab "] offset:%[off]\n\t"
#define EBIC_LOAD_FIRST EBIC_LOAD2("r0", "r1", "a2", "a3")
#define EBIC_WINDOW(X0, X1, X2, X3, X4, X5)                                    \
    EBIC_LOAD2("r2", "r3", "a4", "a5")                                         \
    "s_waitcnt lgkmcnt(2)\n\t"                                                 \
    EBIC_CMP2("r0", "r1", "prev", X0, X1)                                      \
    "s_cbranch_execz 1f\n\t"                                                   \
    "s_cmp_le_i32 %[last], 3\n\t"                                              \
    "s_cbranch_scc1 1f\n\t"                                                    \
    EBIC_LOAD2("r4", "r5", "a6", "a7")                                         \
    "s_waitcnt lgkmcnt(2)\n\t"                                                 \
    EBIC_CMP2("r2", "r3", "r1", X2, X3)                                        \
    "s_cbranch_execz 1f\n\t"                                                   \
    "s_cmp_le_i32 %[last], 5\n\t"                                              \
    "s_cbranch_scc1 1f\n\t"                                                    \
    "s_waitcnt lgkmcnt(0)\n\t"                                                 \
    EBIC_CMP2("r4", "r5", "r3", X4, X5)                                        \
    "1:\n\t"                                                                   \
    "s_waitcnt lgkmcnt(0)\n\t"
#define EBIC_WINDOW_FLIP                                                       \
    EBIC_WINDOW(EBIC_XOR("r0"), EBIC_XOR("r1"), EBIC_XOR("r2"), EBIC_XOR("r3"), \
                EBIC_XOR("r4"), EBIC_XOR("r5"))
#define EBIC_WINDOW_PLAIN EBIC_WINDOW("", "", "", "", "", "")
#define EBIC_SCRATCH_OUTPUTS                                                   \
    [r0] "=&v"(r[0]), [r1] "=&v"(r[1]), [r2] "=&v"(r[2]), [r3] "=&v"(r[3]),    \
        [r4] "=&v"(r[4]), [r5] "=&v"(r[5])
#define EBIC_WINDOW_INPUTS                                                     \
    [last] "s"(last), [a2] "v"(a[2]), [a3] "v"(a[3]), [a4] "v"(a[4]),          \
        [a5] "v"(a[5]), [a6] "v"(a[6]), [a7] "v"(a[7]), [off] "i"(OFF)

// First pair of both chains (values v0, v1 of columns 0 and 1, loaded by
// the caller) and the window, on one 64-row sub-tile; rows outside `valid`
// take no part. Returns the rows still on their chain after column
// min(last, 7); `fall` receives the rows with v1 < v0 (on the <= chain),
// `tie` those with v1 == v0 (still on both), `flip` the per-row sign flip,
// `lastf` the flipped value of column 7 (meaningful when the window ran to
// its end).
template <int OFF>
__device__ __forceinline__ uint64_t subtile_neg(uint64_t valid, int32_t last, const uint32_t (&a)[kWin],
                                                uint32_t sign, float v0, float v1, uint64_t &fall,
                                                uint64_t &tie, uint32_t &flip, float &lastf)
{
    uint64_t out, save, f, t;
    float prev, r[6];
    uint32_t fl;
    asm volatile(
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_mov_b64 %[save], exec\n\t"
        "s_and_b64 exec, exec, %[valid]\n\t"
        EBIC_LOAD_FIRST
        "v_cmp_lt_f32_e64 %[f], %[v1], %[v0]\n\t"
        "v_cmp_eq_f32_e64 %[t], %[v1], %[v0]\n\t"
        "v_cmp_o_f32 vcc, %[v1], %[v0]\n\t"
        "s_nop 4\n\t"  // wait states before a VALU reads an SGPR mask a VALU wrote
        "v_cndmask_b32_e64 %[flip], 0, %[sign], %[f]\n\t"
        "s_and_b64 exec, exec, vcc\n\t"
        "v_xor_b32 %[prev], %[v1], %[flip]\n\t"
        "s_cmp_lt_i32 %[last], 2\n\t"
        "s_cbranch_scc1 1f\n\t"
        EBIC_WINDOW_FLIP
        "1:\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_mov_b64 %[out], exec\n\t"
        "s_mov_b64 exec, %[save]"
        : [out] "=&s"(out), [save] "=&s"(save), [f] "=&s"(f), [t] "=&s"(t), [flip] "=&v"(fl),
          [prev] "=&v"(prev), EBIC_SCRATCH_OUTPUTS
        : [valid] "s"(valid), [v0] "v"(v0), [v1] "v"(v1), [sign] "v"(sign), EBIC_WINDOW_INPUTS
        : "vcc", "scc", "memory");
    fall = f;
    tie = t;
    flip = fl;
    lastf = r[5];
    return out;
}

// The same for the >= chain alone (negative trends not requested).
template <int OFF>
__device__ __forceinline__ uint64_t subtile_pos(uint64_t valid, int32_t last, const uint32_t (&a)[kWin],
                                                float v0, float v1, float &lastf)
{
    uint64_t out, save;
    float r[6];
    asm volatile(
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_mov_b64 %[save], exec\n\t"
        "s_and_b64 exec, exec, %[valid]\n\t"
        EBIC_LOAD_FIRST
        "v_cmp_ge_f32 vcc, %[prev], %[v0]\n\t"
        "s_and_b64 exec, exec, vcc\n\t"
        "s_cmp_lt_i32 %[last], 2\n\t"
        "s_cbranch_scc1 1f\n\t"
        EBIC_WINDOW_PLAIN
        "1:\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_mov_b64 %[out], exec\n\t"
        "s_mov_b64 exec, %[save]"
        : [out] "=&s"(out), [save] "=&s"(save), EBIC_SCRATCH_OUTPUTS
        : [valid] "s"(valid), [v0] "v"(v0), [prev] "v"(v1), EBIC_WINDOW_INPUTS
        : "vcc", "scc", "memory");
    lastf = r[5];
    return out;
}

// The <= chain of the rows tied on the first pair: every value flipped.
template <int OFF>
__device__ __forceinline__ uint64_t subtile_tie(uint64_t tie, int32_t last, const uint32_t (&a)[kWin],
                                                uint32_t sign, float v1, float &lastf)
{
    uint64_t out, save;
    float r[6];
    const float prev = flipped(v1, kSign);
    asm volatile(
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_mov_b64 %[save], exec\n\t"
        "s_and_b64 exec, exec, %[tie]\n\t"
        "s_cbranch_execz 1f\n\t"
        EBIC_LOAD_FIRST
        EBIC_WINDOW_FLIP
        "1:\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_mov_b64 %[out], exec\n\t"
        "s_mov_b64 exec, %[save]"
        : [out] "=&s"(out), [save] "=&s"(save), EBIC_SCRATCH_OUTPUTS
        : [tie] "s"(tie), [prev] "v"(prev), [flip] "v"(sign), EBIC_WINDOW_INPUTS
        : "vcc", "scc", "memory");
    lastf = r[5];
    return out;
}

// Plain-code twin of the three sequences above, with the same exit points;
// it counts the compare instructions it executes (the measurement variant).
struct SubtileRef {
    const unsigned char *tile;
    uint32_t tile_lds;
    int off;
    const uint32_t *a;
    uint64_t *steps;
    __device__ float ld(int u) const
    {
        return *reinterpret_cast<const float *>(tile + (a[u] - tile_lds) + off);
    }
    // Window steps 2..min(last, 7) of a chain whose rows are `alive`.
    __device__ uint64_t window(uint64_t alive, int32_t last, uint32_t flip, float prev, float &lastf) const
    {
#pragma unroll
        for (int u = 2; u < kWin; u += 2) {
            if (alive == 0) break;
            const float x = flipped(ld(u), flip), y = flipped(ld(u + 1), flip);
            alive &= __ballot(x >= prev);
            alive &= __ballot(y >= x);
            *steps += 2;
            prev = y;
            if (alive == 0 || last <= u + 1) break;
        }
        lastf = prev;
        return alive;
    }
};

// Columns kWin..last of a chain (long individuals; rarely any row is left).
__device__ __forceinline__ uint64_t chain_tail(uint64_t alive, int32_t last,
                                               const unsigned char *__restrict__ tile, int off,
                                               const int32_t *__restrict__ c, int cb, int lane4,
                                               uint32_t flip, float prevf, uint64_t &steps,
                                               bool count)
{
    float prev = prevf;
    for (int32_t u = kWin; u <= last && alive; ++u) {
        const float v = flipped(*reinterpret_cast<const float *>(tile + c[u] * cb + lane4 + off), flip);
        alive &= __ballot(v >= prev);
        prev = v;
        if (count) steps += 1;
    }
    return alive;
}

// One individual on one LDS-staged 64-row sub-tile S (v0, v1: this lane's
// values of columns 0 and 1): its matched rows M and negative-only rows G.
template <int L, int S, bool NEG, bool COUNT>
__device__ __forceinline__ void eval_subtile(const unsigned char *__restrict__ tile, uint32_t tile_lds,
                                             const uint32_t (&a)[kWin], const int32_t *__restrict__ c,
                                             int32_t last, int lane4, uint64_t valid, float v0,
                                             float v1, uint64_t &M, uint64_t &G, uint64_t &steps)
{
    constexpr int CB = L * kWave * 4;
    constexpr int OFF = S * kWave * 4;
    if (last == 0) {  // one column: the row counts unless its value is missing
        M = __ballot(v0 == v0) & valid;
        G = 0;
        if (COUNT) steps += 1;
        return;
    }
    if constexpr (NEG) {
        uint64_t fall, tie, out;
        float lastf;
        uint32_t flip;
        if constexpr (COUNT) {
            const SubtileRef r{tile, tile_lds, OFF, a, &steps};
            fall = __ballot(v1 < v0) & valid;
            tie = __ballot(v1 == v0) & valid;
            flip = v1 < v0 ? kSign : 0u;
            steps += 3;
            out = __ballot(v1 == v1 && v0 == v0) & valid;
            lastf = flipped(v1, flip);
            if (last >= 2) out = r.window(out, last, flip, lastf, lastf);
        } else {
            out = subtile_neg<OFF>(valid, last, a, kSign, v0, v1, fall, tie, flip, lastf);
        }
        if (last >= kWin && out) out = chain_tail(out, last, tile, OFF, c, CB, lane4, flip, lastf, steps, COUNT);
        uint64_t m = out, g = out & fall;
        if (tie) {
            uint64_t tout = tie;
            if (last >= 2) {
                float tl;
                if constexpr (COUNT) {
                    const SubtileRef r{tile, tile_lds, OFF, a, &steps};
                    tout = r.window(tie, last, kSign, flipped(v1, kSign), tl);
                } else {
                    tout = subtile_tie<OFF>(tie, last, a, kSign, v1, tl);
                }
                if (last >= kWin && tout)
                    tout = chain_tail(tout, last, tile, OFF, c, CB, lane4, kSign, tl, steps, COUNT);
            }
            m |= tout;
            g |= tout & ~out;
        }
        M = m;
        G = g;
    } else {
        uint64_t out;
        float lastf;
        if constexpr (COUNT) {
            const SubtileRef r{tile, tile_lds, OFF, a, &steps};
            out = __ballot(v1 >= v0) & valid;
            steps += 1;
            lastf = v1;
            if (last >= 2) out = r.window(out, last, 0u, lastf, lastf);
        } else {
            out = subtile_pos<OFF>(valid, last, a, v0, v1, lastf);
        }
        if (last >= kWin && out) out = chain_tail(out, last, tile, OFF, c, CB, lane4, 0u, lastf, steps, COUNT);
        M = out;
        G = 0;
    }
}

// One individual on the L LDS-staged sub-tiles of a chunk, one sub-tile at a
// time (each with its own early exit).
template <int L, bool NEG, bool COUNT>
__device__ __forceinline__ void eval_lds(const unsigned char *__restrict__ tile, int32_t last,
                                         const int32_t *__restrict__ c, const int4 &w03,
                                         const int4 &w47, int lane4, const uint64_t (&valid)[L],
                                         uint64_t (&M)[L], uint64_t (&G)[L], uint64_t &steps)
{
    constexpr int CB = L * kWave * 4;  // bytes of one staged column
    const uint32_t tile_lds = lds_addr(tile);
    const uint32_t base = tile_lds + lane4;
    const int32_t w[kWin] = {w03.x, w03.y, w03.z, w03.w, w47.x, w47.y, w47.z, w47.w};
    uint32_t a[kWin];
#pragma unroll
    for (int u = 0; u < kWin; ++u) a[u] = base + w[u] * CB;
    // The first pair of every sub-tile is loaded up front, so only the first
    // sub-tile waits for it.
    float v0[L], v1[L];
#pragma unroll
    for (int s = 0; s < L; ++s) {
        v0[s] = *reinterpret_cast<const float *>(tile + (a[0] - tile_lds) + s * kWave * 4);
        v1[s] = *reinterpret_cast<const float *>(tile + (a[1] - tile_lds) + s * kWave * 4);
    }
    eval_subtile<L, 0, NEG, COUNT>(tile, tile_lds, a, c, last, lane4, valid[0], v0[0], v1[0], M[0], G[0], steps);
    if constexpr (L > 1)
        eval_subtile<L, 1, NEG, COUNT>(tile, tile_lds, a, c, last, lane4, valid[1], v0[1], v1[1], M[1], G[1], steps);
    if constexpr (L > 2) {
        eval_subtile<L, 2, NEG, COUNT>(tile, tile_lds, a, c, last, lane4, valid[2], v0[2], v1[2], M[2], G[2], steps);
        eval_subtile<L, 3, NEG, COUNT>(tile, tile_lds, a, c, last, lane4, valid[3], v0[3], v1[3], M[3], G[3], steps);
    }
}

// ---------------------------------------------------------------------------
// L sub-tiles interleaved (L = 2 or 4): one instruction stream evaluates the
// same individual on all L sub-tiles of the chunk, each with its own alive
// mask in scalar registers, so the compares of different sub-tiles are
// independent and hide each other's latency. Column u of sub-tile s of this
// lane sits at base + u*CB + s*256 bytes, one address per column.
//
// Register rotation: column u is loaded into set u mod 3; while column u is
// compared (against set (u-1) mod 3) the loads of column u+1 are in flight.
// Window columns past the last one repeat the last column (the header clamps
// them), and a repeated column never removes a row (x >= x for every non-NaN
// x; NaN rows are already gone), so the window may run past `last` without
// changing the result; the exits after columns 3 and 5 only save work.
// ---------------------------------------------------------------------------
#define IL_T "f32"
#define IL_LD "ds_read_b32"
#define IL_O1 "256"
#define IL_O2 "512"
#define IL_O3 "768"
#define IL_SH4 "10"
#define IL_SH2 "9"
#define IL_NAME(f) f##_f32
#include "ebic_chain.inc"
#undef IL_T
#undef IL_LD
#undef IL_O1
#undef IL_O2
#undef IL_O3
#undef IL_SH4
#undef IL_SH2
#undef IL_NAME

#define IL_T "f16"
#define IL_LD "ds_read_u16"
#define IL_O1 "128"
#define IL_O2 "256"
#define IL_O3 "384"
#define IL_SH4 "9"
#define IL_SH2 "8"
#define IL_NAME(f) f##_f16
#include "ebic_chain.inc"
#undef IL_T
#undef IL_LD
#undef IL_O1
#undef IL_O2
#undef IL_O3
#undef IL_SH4
#undef IL_SH2
#undef IL_NAME

// One staged element as a float: an FP32 value, or an FP16 rank code
// (converted exactly; NaN stays NaN).
template <typename E>
__device__ __forceinline__ float lds_val(const unsigned char *p)
{
    if constexpr (std::is_same<E, float>::value) return *reinterpret_cast<const float *>(p);
    else return __half2float(__ushort_as_half(*reinterpret_cast<const uint16_t *>(p)));
}

// Plain-code twin of the interleaved window (the measurement variant and the
// rare paths): same exit points as the sequences above. `prev` holds the
// flipped values of column 1; counts executed compare instructions. `flip`
// is the FP32 sign bit or 0 (values are compared as floats here).
template <int L, bool COUNT, typename E>
__device__ __forceinline__ void il_window_ref(const unsigned char *__restrict__ base, const int32_t (&w)[kWin],
                                              int32_t last, const uint32_t (&flip)[L], float (&prev)[L],
                                              uint64_t (&alive)[L], uint64_t &steps)
{
    constexpr int SB = kWave * (int)sizeof(E), CB = L * SB;
#pragma unroll
    for (int u = 2; u < kWin; ++u) {
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const float y = flipped(lds_val<E>(base + w[u] * CB + s * SB), flip[s]);
            alive[s] &= __ballot(y >= prev[s]);
            prev[s] = y;
        }
        if (COUNT) steps += L;
        if (u == 3 || u == 5) {
            uint64_t any = 0;
#pragma unroll
            for (int s = 0; s < L; ++s) any |= alive[s];
            if (any == 0 || last <= u) return;
        }
    }
}

// Columns kWin..last (long individuals; rarely any row is left).
template <int L, bool COUNT, typename E>
__device__ __forceinline__ void il_tail(const unsigned char *__restrict__ base, const int32_t *__restrict__ c,
                                        int32_t last, const uint32_t (&flip)[L], float (&prev)[L],
                                        uint64_t (&alive)[L], uint64_t &steps)
{
    constexpr int SB = kWave * (int)sizeof(E), CB = L * SB;
    for (int32_t u = kWin; u <= last; ++u) {
        const int32_t col = c[u];
        uint64_t any = 0;
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const float y = flipped(lds_val<E>(base + col * CB + s * SB), flip[s]);
            alive[s] &= __ballot(y >= prev[s]);
            prev[s] = y;
            any |= alive[s];
        }
        if (COUNT) steps += L;
        if (any == 0) return;
    }
}

// One individual on the L (2 or 4) sub-tiles of a chunk, staged as FP32
// values (E = float) or FP16 rank codes (E = uint16_t). Rows outside the
// matrix hold NaN in the tile, so they never match.
template <int L, bool NEG, bool COUNT, typename E>
__device__ __forceinline__ void eval_lds_il(const unsigned char *__restrict__ tile, int32_t last,
                                            const int32_t *__restrict__ c, const int4 &w03,
                                            const int4 &w47, int lane, uint64_t (&M)[L],
                                            uint64_t (&G)[L], uint64_t &steps)
{
    static_assert(L == 2 || L == 4, "interleaved evaluation takes 2 or 4 sub-tiles");
    constexpr bool H = !std::is_same<E, float>::value;
    constexpr int SB = kWave * (int)sizeof(E), CB = L * SB;
    const unsigned char *base = tile + lane * (int)sizeof(E);
    const int32_t w[kWin] = {w03.x, w03.y, w03.z, w03.w, w47.x, w47.y, w47.z, w47.w};
    auto ld = [&](int32_t col, int s) -> float { return lds_val<E>(base + col * CB + s * SB); };
    if (last == 0) {  // one column: the row counts unless its value is missing
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const float v = ld(w[0], s);
            M[s] = __ballot(v == v);
            G[s] = 0;
        }
        if (COUNT) steps += L;
        return;
    }
    uint64_t A[L], F[L], T = 0;
    uint32_t f[L];
    if constexpr (COUNT || !NEG) {
        float prev[L];
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const float v0 = ld(w[0], s), v1 = ld(w[1], s);
            if constexpr (NEG) {
                F[s] = __ballot(v1 < v0);
                A[s] = __ballot(!__builtin_isunordered(v1, v0));
                T |= __ballot(v1 == v0);
                f[s] = v1 < v0 ? kSign : 0u;
            } else {
                F[s] = 0;
                A[s] = __ballot(v1 >= v0);
                f[s] = 0u;
            }
            prev[s] = flipped(v1, f[s]);
        }
        if (COUNT) steps += (NEG ? 3 : 1) * L;
        if constexpr (COUNT) {
            if (last >= 2) il_window_ref<L, COUNT, E>(base, w, last, f, prev, A, steps);
        } else {
            const uint32_t b = lds_addr(base);
            if constexpr (H) {
                if constexpr (L == 4) il_pos4_f16(b, w, last, A);
                else il_pos2_f16(b, w, last, A);
            } else {
                if constexpr (L == 4) il_pos4_f32(b, w, last, A);
                else il_pos2_f32(b, w, last, A);
            }
        }
    } else {
        const uint32_t b = lds_addr(base);
        if constexpr (H) {
            // The FP16 sign bit flips a code; the plain code below compares
            // converted floats, so the flips are widened afterwards.
            if constexpr (L == 4) il_neg4_f16(b, w, last, kSign >> 16, A, F, T, f);
            else il_neg2_f16(b, w, last, kSign >> 16, A, F, T, f);
#pragma unroll
            for (int s = 0; s < L; ++s) f[s] <<= 16;
        } else {
            if constexpr (L == 4) il_neg4_f32(b, w, last, kSign, A, F, T, f);
            else il_neg2_f32(b, w, last, kSign, A, F, T, f);
        }
    }
    if (last >= kWin) {
        uint64_t any = 0;
#pragma unroll
        for (int s = 0; s < L; ++s) any |= A[s];
        if (any) {
            float prev[L];
#pragma unroll
            for (int s = 0; s < L; ++s) prev[s] = flipped(ld(w[kWin - 1], s), f[s]);
            il_tail<L, COUNT, E>(base, c, last, f, prev, A, steps);
        }
    }
#pragma unroll
    for (int s = 0; s < L; ++s) {
        M[s] = A[s];
        if constexpr (NEG && !COUNT)  // on the scalar unit (wave-uniform masks)
            asm("s_and_b64 %0, %1, %2" : "=s"(G[s]) : "s"(A[s]), "s"(F[s]) : "scc");
        else
            G[s] = A[s] & F[s];
    }
    if constexpr (NEG) {
        if (T && last >= 2) {
            // Rows tied on the first pair also try the <= chain.
            uint64_t ta[L];
            uint32_t fl[L];
            float prev[L];
#pragma unroll
            for (int s = 0; s < L; ++s) {
                const float v0 = ld(w[0], s), v1 = ld(w[1], s);
                ta[s] = __ballot(v1 == v0);
                fl[s] = kSign;
                prev[s] = flipped(v1, kSign);
            }
            if (COUNT) steps += L;
            if (last >= 2) il_window_ref<L, COUNT, E>(base, w, last, fl, prev, ta, steps);
            if (last >= kWin) {
                uint64_t any = 0;
#pragma unroll
                for (int s = 0; s < L; ++s) any |= ta[s];
                if (any) {
#pragma unroll
                    for (int s = 0; s < L; ++s) prev[s] = flipped(ld(w[kWin - 1], s), kSign);
                    il_tail<L, COUNT, E>(base, c, last, fl, prev, ta, steps);
                }
            }
#pragma unroll
            for (int s = 0; s < L; ++s) {
                M[s] |= ta[s];
                G[s] |= ta[s] & ~A[s];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Byte rank codes: four sub-tiles in one 32-bit word per lane.
//
// Byte b of lane l's word is the code (0..127) of row 64*b + l of the staged
// 256-row chunk, and codes order exactly as the values do. For codes x and
// y below 128, the 32-bit difference (x | 0x80808080) - y never borrows
// across bytes (every byte of it lies in [1, 255]), and bit 7 of a byte is
// set exactly when that byte's x >= y: one subtraction compares four rows.
// A row that falls on the first pair has its codes mirrored (t ^ 0x7F
// reverses their order), so every row again follows one >= chain, of
// oriented codes x_j = t_j ^ fm. With fH = fm | 0x80808080, nf = ~fm and
// nx = -x_{j-1}, one column is
//   D = (t_j ^ fH) + nx      = (x_j | 0x80808080) - x_{j-1}
//   nx = (t_j ^ nf) + 1      = -x_j
// and every two columns alive &= D_j & D_{j+1} (one three-input AND):
// five VALU operations per two columns of 256 rows. `alive` keeps bit 7 of
// the bytes of the rows still on their chain (it starts from the in-range
// rows). Rows tied on the first pair then run the <= chain on their own:
// every code mirrored, fH = 0xFFFFFFFF, nf = 0x80808080. The same sequences
// run on 16-bit parts (codes below 2^15, two rows per word: rows l and
// 64 + l of a 128-row group) with the constants of Lanes<16>.
// ---------------------------------------------------------------------------
// Lane parts of BITS bits (codes below 2^(BITS-1)): the constants of the
// arithmetic above.
template <int BITS> struct Lanes;
template <> struct Lanes<8> {
    static constexpr uint32_t H = 0x80808080u;    // the top bit of every part
    static constexpr uint32_t TWO = 0x01010100u;  // D + E, summed over the parts
    static constexpr uint32_t MIR = 0x7f7f7f7fu;  // mirrors every part
    static constexpr int SHF = 7;                 // top bit -> bit 0 of its part
    static constexpr int PARTS = 4;               // rows per word
};
template <> struct Lanes<16> {
    static constexpr uint32_t H = 0x80008000u;
    static constexpr uint32_t TWO = 0x00010000u;
    static constexpr uint32_t MIR = 0x7fff7fffu;
    static constexpr int SHF = 15;
    static constexpr int PARTS = 2;
};
// Three parts of ten bits (bits 30-31 unused; codes below 2^9): the same
// arithmetic holds per part, and the sum D + E of the first pair carries
// into bits 10, 20 and 30.
template <> struct Lanes<10> {
    static constexpr uint32_t H = 0x20080200u;
    static constexpr uint32_t TWO = 0x40100400u;
    static constexpr uint32_t MIR = 0x1ff7fdffu;
    static constexpr int SHF = 9;
    static constexpr int PARTS = 3;
};


#define BY_LOAD(t, w)                                                          \
    "v_lshl_add_u32 %[ad], %[" w "], %[sh], %[base]\n\t"                       \
    "ds_read_b32 %[" t "], %[ad]\n\t"
#define BY_PAIR(ta, tb, FH, NF, NX, AL, ALIN)                                  \
    "v_xad_u32 %[D], %[" ta "], " FH ", %[" NX "]\n\t"                         \
    "v_xad_u32 %[" NX "], %[" ta "], " NF ", 1\n\t"                            \
    "v_xad_u32 %[D2], %[" tb "], " FH ", %[" NX "]\n\t"                        \
    "v_xad_u32 %[" NX "], %[" tb "], " NF ", 1\n\t"                            \
    "v_bitop3_b32 %[" AL "], %[" ALIN "], %[D], %[D2] bitop3:0x80\n\t"
// The window's last pair: no reference is carried past column 7 (the
// columns after the window start again from column 7).
#define BY_PAIR_LAST(ta, tb, FH, NF, NX, AL, ALIN)                             \
    "v_xad_u32 %[D], %[" ta "], " FH ", %[" NX "]\n\t"                         \
    "v_xad_u32 %[" NX "], %[" ta "], " NF ", 1\n\t"                            \
    "v_xad_u32 %[D2], %[" tb "], " FH ", %[" NX "]\n\t"                        \
    "v_bitop3_b32 %[" AL "], %[" ALIN "], %[D], %[D2] bitop3:0x80\n\t"
// After column 3 only the length ends the chain (256 rows rarely all fail
// within four columns); after column 5 also the rows left.
#define BY_EXIT_LAST(u, L) "s_cmp_le_i32 %[last], " u "\n\t" "s_cbranch_scc1 " L "\n\t"
#define BY_EXIT(u, AL, L)                                                      \
    "v_cmp_ne_u32_e64 %[tmp], 0, %[" AL "]\n\t"                                \
    "s_cmp_lg_u64 %[tmp], 0\n\t"                                               \
    "s_cbranch_scc0 " L "\n\t" BY_EXIT_LAST(u, L)
// Columns 2..7: t2 and t3 hold (or are loading) columns 2 and 3; loads run
// two columns ahead. Window columns past the last one repeat it, which
// changes nothing. The first pair's AND reads the rows from ALIN.
#define BY_WINDOW(FH, NF, NX, AL, ALIN, L)                                     \
    BY_LOAD("t0", "w4") BY_LOAD("t1", "w5") "s_waitcnt lgkmcnt(2)\n\t"         \
    BY_PAIR("t2", "t3", FH, NF, NX, AL, ALIN) BY_EXIT_LAST("3", L)             \
    BY_LOAD("t2", "w6") BY_LOAD("t3", "w7") "s_waitcnt lgkmcnt(2)\n\t"         \
    BY_PAIR("t0", "t1", FH, NF, NX, AL, AL) BY_EXIT("5", AL, L)                \
    "s_waitcnt lgkmcnt(0)\n\t" BY_PAIR_LAST("t2", "t3", FH, NF, NX, AL, AL)
#define BY_SCRATCH                                                             \
    [t0] "=&v"(t0), [t1] "=&v"(t1), [t2] "=&v"(t2), [t3] "=&v"(t3), [ad] "=&v"(ad), \
        [D] "=&v"(D), [D2] "=&v"(D2), [tmp] "=&s"(tmp)
#define BY_COLS                                                                \
    [base] "v"(base), [w0] "s"(w[0]), [w1] "s"(w[1]), [w2] "s"(w[2]), [w3] "s"(w[3]), \
        [w4] "s"(w[4]), [w5] "s"(w[5]), [w6] "s"(w[6]), [w7] "s"(w[7]), [last] "s"(last), \
        [sh] "i"(SH), [H] "i"(T::H), [TWO] "i"(T::TWO), [SHF] "i"(T::SHF)

// The sequences below take SH = log2 of the bytes one staged column
// occupies (8: 256-row chunks, 9: 512-row chunks of two 256-row groups).

// Both chains through column min(last, 7): alive (rows on their oriented
// chain), fall (bit 7 of the in-range rows with t1 < t0) and tied (the
// rows tied on the first pair that also follow the <= chain; 0 unless
// last >= 2). The sequence starts with lgkmcnt(0) (no scalar load in
// flight, so LDS operations complete in issue order and lgkmcnt(n) means
// that all but the last n issued are done) and ends with it.
template <int SH, int BITS = 8, bool TIES = true>
__device__ __forceinline__ void by_neg(uint32_t base, const int32_t (&w)[kWin], int32_t last, uint32_t hv,
                                       uint32_t &alive, uint32_t &fall, uint32_t &tied)
{
    using T = Lanes<BITS>;
    uint32_t t0, t1, t2, t3, ad, D, D2, fm, fH, nf, nx;
    uint64_t tmp, tany;
    if constexpr (!TIES) {
        // No row of the chunk holds two equal values: a row falls exactly
        // when it does not rise, and no row is tied.
        asm volatile(
            "s_waitcnt lgkmcnt(0)\n\t"
            BY_LOAD("t0", "w0") BY_LOAD("t1", "w1") BY_LOAD("t2", "w2") BY_LOAD("t3", "w3")
            "s_waitcnt lgkmcnt(2)\n\t"
            "v_or_b32_e32 %[D], %[H], %[t1]\n\t"
            "v_sub_u32_e32 %[D], %[D], %[t0]\n\t"           // top bits: t1 >= t0
            "v_bfi_b32 %[fall], %[D], 0, %[hv]\n\t"         // ~D & hv: falling, in range
            "v_lshrrev_b32_e32 %[fm], %[SHF], %[fall]\n\t"
            "v_sub_u32_e32 %[fm], %[fall], %[fm]\n\t"       // all low bits of each falling part
            "v_or_b32_e32 %[fH], %[H], %[fm]\n\t"
            "v_not_b32_e32 %[nf], %[fm]\n\t"
            "v_xad_u32 %[nx], %[t1], %[nf], 1\n\t"
            "s_cmp_lt_i32 %[last], 2\n\t"
            "s_cbranch_scc1 6f\n\t"
            BY_WINDOW("%[fH]", "%[nf]", "nx", "alive", "hv", "2f")
            "2:\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            "s_branch 5f\n\t"
            "6:\n\t"  // two columns: every row in range is on its chain
            "v_mov_b32_e32 %[alive], %[hv]\n\t"
            "5:"
            : BY_SCRATCH, [fm] "=&v"(fm), [fH] "=&v"(fH), [nf] "=&v"(nf), [nx] "=&v"(nx),
              [alive] "=&v"(alive), [fall] "=&v"(fall)
            : BY_COLS, [hv] "v"(hv)
            : "scc", "memory");
        tied = 0;
        return;
    }
    asm volatile(
        "s_waitcnt lgkmcnt(0)\n\t"
        BY_LOAD("t0", "w0") BY_LOAD("t1", "w1") BY_LOAD("t2", "w2") BY_LOAD("t3", "w3")
        "s_waitcnt lgkmcnt(2)\n\t"
        "v_or_b32_e32 %[D], %[H], %[t1]\n\t"
        "v_sub_u32_e32 %[D], %[D], %[t0]\n\t"           // top bits: t1 >= t0
        "v_sub_u32_e32 %[D2], %[TWO], %[D]\n\t"         // = (t0 | H) - t1, top bits: t0 >= t1
        "v_bitop3_b32 %[tied], %[D], %[D2], %[hv] bitop3:0x80\n\t"  // tied, in range
        "v_bitop3_b32 %[fall], %[D], %[D2], %[hv] bitop3:0x08\n\t"  // ~D & D2 & hv: falling
        "v_lshrrev_b32_e32 %[fm], %[SHF], %[fall]\n\t"
        "v_sub_u32_e32 %[fm], %[fall], %[fm]\n\t"       // all low bits of each falling part
        "v_or_b32_e32 %[fH], %[H], %[fm]\n\t"
        "v_not_b32_e32 %[nf], %[fm]\n\t"
        "v_xad_u32 %[nx], %[t1], %[nf], 1\n\t"
        "v_cmp_ne_u32_e64 %[tany], 0, %[tied]\n\t"
        "s_cmp_lt_i32 %[last], 2\n\t"
        "s_cbranch_scc1 6f\n\t"
        BY_WINDOW("%[fH]", "%[nf]", "nx", "alive", "hv", "2f")
        "2:\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        // The rows tied on the first pair: the <= chain from column 1.
        "s_cmp_lg_u64 %[tany], 0\n\t"
        "s_cbranch_scc0 4f\n\t"
        BY_LOAD("t1", "w1") BY_LOAD("t2", "w2") BY_LOAD("t3", "w3")
        "s_waitcnt lgkmcnt(2)\n\t"
        "v_xad_u32 %[nx], %[t1], %[hi], 1\n\t"
        BY_WINDOW("-1", "%[hi]", "nx", "tied", "tied", "3f")
        "3:\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_branch 5f\n\t"
        "6:\n\t"  // two columns: every row in range is on its chain
        "v_mov_b32_e32 %[alive], %[hv]\n\t"
        "4:\n\t"
        "v_mov_b32_e32 %[tied], 0\n\t"
        "5:"
        : BY_SCRATCH, [fm] "=&v"(fm), [fH] "=&v"(fH), [nf] "=&v"(nf), [nx] "=&v"(nx),
          [alive] "=&v"(alive), [fall] "=&v"(fall), [tied] "=&v"(tied), [tany] "=&s"(tany)
        : BY_COLS, [hv] "v"(hv), [hi] "s"(T::H)
        : "scc", "memory");
}

// The >= chain alone through column min(last, 7) (waits as above).
template <int SH, int BITS = 8>
__device__ __forceinline__ void by_pos(uint32_t base, const int32_t (&w)[kWin], int32_t last, uint32_t hv,
                                       uint32_t &alive)
{
    using T = Lanes<BITS>;
    uint32_t t0, t1, t2, t3, ad, D, D2, nx;
    uint64_t tmp;
    asm volatile(
        "s_waitcnt lgkmcnt(0)\n\t"
        BY_LOAD("t0", "w0") BY_LOAD("t1", "w1") BY_LOAD("t2", "w2") BY_LOAD("t3", "w3")
        "s_waitcnt lgkmcnt(2)\n\t"
        "v_or_b32_e32 %[D], %[H], %[t1]\n\t"
        "v_sub_u32_e32 %[D], %[D], %[t0]\n\t"
        "v_and_b32_e32 %[alive], %[D], %[hv]\n\t"
        "v_sub_u32_e32 %[nx], 0, %[t1]\n\t"
        "s_cmp_lt_i32 %[last], 2\n\t"
        "s_cbranch_scc1 2f\n\t"
        BY_WINDOW("%[hi]", "-1", "nx", "alive", "alive", "2f")
        "2:\n\t"
        "s_waitcnt lgkmcnt(0)"
        : BY_SCRATCH, [nx] "=&v"(nx), [alive] "=&v"(alive)
        : BY_COLS, [hv] "v"(hv), [hi] "s"(T::H)
        : "scc", "memory");
}

#undef BY_LOAD
#undef BY_PAIR
#undef BY_PAIR_LAST
#undef BY_EXIT_LAST
#undef BY_EXIT
#undef BY_WINDOW
#undef BY_SCRATCH
#undef BY_COLS

// ---------------------------------------------------------------------------
// Two lane words per chunk: byte codes in 512-row chunks (two 256-row groups,
// four rows per word) or 16-bit codes in 256-row chunks (two 128-row groups,
// two rows per word: lane l's word holds rows l and 64 + l of its group). A
// staged column is 512 bytes in both cases, the second word at +256. Both
// words' chains run in one instruction stream with their operations
// alternating: a column's two words share one address and hide each other's
// latency, and the window ends when no row of either word is left. The
// arithmetic is the byte one above with lane parts of BITS bits (codes below
// 2^(BITS-1)); the reference carried from column to column is
// q = H - x_{j-1} (each part in 1..2^(BITS-1), no borrow), which needs fm and
// nf but not fH:
//   D = (t_j ^ fm) + q       = (x_j | H) - x_{j-1}
//   q = (t_j ^ nf) + H + 1   = H - x_j
// Chunks whose rows hold no two equal values (tie flags computed at upload)
// skip the tie detection and the tie chain.
// ---------------------------------------------------------------------------
#define B2_LOAD(t, w)                                                          \
    "v_lshl_add_u32 %[ad], %[" w "], %[sh2], %[base]\n\t"                      \
    "ds_read_b32 %[" t "a], %[ad]\n\t"                                         \
    "ds_read_b32 %[" t "b], %[ad] offset:256\n\t"
#define B2_PAIR(ta, tb, FMA, FMB, NFA, NFB, AOA, AOB, AIA, AIB)                \
    "v_xad_u32 %[Da], %[" ta "a], " FMA ", %[qa]\n\t"                          \
    "v_xad_u32 %[Db], %[" ta "b], " FMB ", %[qb]\n\t"                          \
    "v_xad_u32 %[qa], %[" ta "a], " NFA ", %[hp]\n\t"                          \
    "v_xad_u32 %[qb], %[" ta "b], " NFB ", %[hp]\n\t"                          \
    "v_xad_u32 %[Ea], %[" tb "a], " FMA ", %[qa]\n\t"                          \
    "v_xad_u32 %[Eb], %[" tb "b], " FMB ", %[qb]\n\t"                          \
    "v_xad_u32 %[qa], %[" tb "a], " NFA ", %[hp]\n\t"                          \
    "v_xad_u32 %[qb], %[" tb "b], " NFB ", %[hp]\n\t"                          \
    "v_bitop3_b32 %[" AOA "], %[" AIA "], %[Da], %[Ea] bitop3:0x80\n\t"        \
    "v_bitop3_b32 %[" AOB "], %[" AIB "], %[Db], %[Eb] bitop3:0x80\n\t"
// The window's last pair: no reference is carried past column 7.
#define B2_PAIR_LAST(ta, tb, FMA, FMB, NFA, NFB, AOA, AOB, AIA, AIB)           \
    "v_xad_u32 %[Da], %[" ta "a], " FMA ", %[qa]\n\t"                          \
    "v_xad_u32 %[Db], %[" ta "b], " FMB ", %[qb]\n\t"                          \
    "v_xad_u32 %[qa], %[" ta "a], " NFA ", %[hp]\n\t"                          \
    "v_xad_u32 %[qb], %[" ta "b], " NFB ", %[hp]\n\t"                          \
    "v_xad_u32 %[Ea], %[" tb "a], " FMA ", %[qa]\n\t"                          \
    "v_xad_u32 %[Eb], %[" tb "b], " FMB ", %[qb]\n\t"                          \
    "v_bitop3_b32 %[" AOA "], %[" AIA "], %[Da], %[Ea] bitop3:0x80\n\t"        \
    "v_bitop3_b32 %[" AOB "], %[" AIB "], %[Db], %[Eb] bitop3:0x80\n\t"
#define B2_EXIT_LAST(u, L) "s_cmp_le_i32 %[last], " u "\n\t" "s_cbranch_scc1 " L "\n\t"
#define B2_EXIT(u, AA, AB, L)                                                  \
    "v_or_b32_e32 %[Da], %[" AA "], %[" AB "]\n\t"                             \
    "v_cmp_ne_u32_e64 %[tmp], 0, %[Da]\n\t"                                    \
    "s_cmp_lg_u64 %[tmp], 0\n\t"                                               \
    "s_cbranch_scc0 " L "\n\t" B2_EXIT_LAST(u, L)
// Columns 2..7 (t2, t3 hold or are loading columns 2 and 3; loads run two
// columns ahead; two loads per column).
#define B2_WINDOW(FMA, FMB, NFA, NFB, AA, AB, IA, IB, L)                       \
    B2_LOAD("t0", "w4") B2_LOAD("t1", "w5") "s_waitcnt lgkmcnt(4)\n\t"         \
    B2_PAIR("t2", "t3", FMA, FMB, NFA, NFB, AA, AB, IA, IB)                    \
    B2_EXIT_LAST("3", L)                                                       \
    B2_LOAD("t2", "w6") B2_LOAD("t3", "w7") "s_waitcnt lgkmcnt(4)\n\t"         \
    B2_PAIR("t0", "t1", FMA, FMB, NFA, NFB, AA, AB, AA, AB)                    \
    B2_EXIT("5", AA, AB, L)                                                    \
    "s_waitcnt lgkmcnt(0)\n\t"                                                 \
    B2_PAIR_LAST("t2", "t3", FMA, FMB, NFA, NFB, AA, AB, AA, AB)
#define B2_SCRATCH                                                             \
    [t0a] "=&v"(t0a), [t0b] "=&v"(t0b), [t1a] "=&v"(t1a), [t1b] "=&v"(t1b),    \
        [t2a] "=&v"(t2a), [t2b] "=&v"(t2b), [t3a] "=&v"(t3a), [t3b] "=&v"(t3b), \
        [ad] "=&v"(ad), [Da] "=&v"(Da), [Db] "=&v"(Db), [Ea] "=&v"(Ea), [Eb] "=&v"(Eb), \
        [qa] "=&v"(qa), [qb] "=&v"(qb), [tmp] "=&s"(tmp)
#define B2_COLS                                                                \
    [base] "v"(base), [w0] "s"(w[0]), [w1] "s"(w[1]), [w2] "s"(w[2]), [w3] "s"(w[3]), \
        [w4] "s"(w[4]), [w5] "s"(w[5]), [w6] "s"(w[6]), [w7] "s"(w[7]), [last] "s"(last), \
        [hp] "s"(T::H + 1u), [H] "i"(T::H), [TWO] "i"(T::TWO), [SHF] "i"(T::SHF), [MIR] "i"(T::MIR), \
        [sh2] "i"(SH)
// First pair of a word (X = a or b); the two words' operations alternate.
// D: top bit of a part where t1 >= t0; E: where t0 >= t1 (tie test only).
#define B2_F1(X) "v_or_b32_e32 %[D" X "], %[H], %[t1" X "]\n\t"
#define B2_F2(X) "v_sub_u32_e32 %[D" X "], %[D" X "], %[t0" X "]\n\t"
#define B2_F3(X) "v_sub_u32_e32 %[E" X "], %[TWO], %[D" X "]\n\t"
#define B2_F4(X) "v_bitop3_b32 %[tied" X "], %[D" X "], %[E" X "], %[hv" X "] bitop3:0x80\n\t"
#define B2_F5(X) "v_bfi_b32 %[fall" X "], %[D" X "], 0, %[hv" X "]\n\t"
#define B2_F6(X) "v_lshrrev_b32_e32 %[E" X "], %[SHF], %[fall" X "]\n\t"
#define B2_F7(X) "v_sub_u32_e32 %[fm" X "], %[fall" X "], %[E" X "]\n\t"
#define B2_F8(X) "v_not_b32_e32 %[nf" X "], %[fm" X "]\n\t"
#define B2_F9(X) "v_xad_u32 %[q" X "], %[t1" X "], %[nf" X "], %[hp]\n\t"
#define B2_AB(F) F("a") F("b")
#define B2_FIRST_TIES                                                          \
    B2_AB(B2_F1) B2_AB(B2_F2) B2_AB(B2_F3) B2_AB(B2_F4) B2_AB(B2_F5)           \
    B2_AB(B2_F6) B2_AB(B2_F7) B2_AB(B2_F8) B2_AB(B2_F9)
#define B2_FIRST_NOTIES                                                        \
    B2_AB(B2_F1) B2_AB(B2_F2) B2_AB(B2_F5) B2_AB(B2_F6) B2_AB(B2_F7)           \
    B2_AB(B2_F8) B2_AB(B2_F9)

// Both chains on both words through column min(last, 7); outputs per word
// as in by_neg (tied = 0 without TIES). Waits count LDS operations; the
// sequence starts and ends with lgkmcnt(0).
// SH: log2 of the bytes one staged column occupies (9: the two words of a
// 512-byte column; 10: a pair of words of a 1024-byte column, the second
// pair at base + 512).
template <int BITS, bool TIES, int SH = 9>
__device__ __forceinline__ void by2_neg(uint32_t base, const int32_t (&w)[kWin], int32_t last, uint32_t hva,
                                        uint32_t hvb, uint32_t &alivea, uint32_t &aliveb, uint32_t &falla,
                                        uint32_t &fallb, uint32_t &tieda, uint32_t &tiedb)
{
    using T = Lanes<BITS>;
    uint32_t t0a, t0b, t1a, t1b, t2a, t2b, t3a, t3b, ad, Da, Db, Ea, Eb, qa, qb, fma, fmb, nfa, nfb;
    uint64_t tmp, tany;
    if constexpr (TIES) {
        asm volatile(
            "s_waitcnt lgkmcnt(0)\n\t"
            B2_LOAD("t0", "w0") B2_LOAD("t1", "w1") B2_LOAD("t2", "w2") B2_LOAD("t3", "w3")
            "s_waitcnt lgkmcnt(4)\n\t"
            B2_FIRST_TIES
            "v_or_b32_e32 %[Da], %[tieda], %[tiedb]\n\t"
            "v_cmp_ne_u32_e64 %[tany], 0, %[Da]\n\t"
            "s_cmp_lt_i32 %[last], 2\n\t"
            "s_cbranch_scc1 6f\n\t"
            B2_WINDOW("%[fma]", "%[fmb]", "%[nfa]", "%[nfb]", "alivea", "aliveb", "hva", "hvb", "2f")
            "2:\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            // The rows tied on the first pair: the <= chain from column 1
            // (every code mirrored: fm = MIR, nf = H).
            "s_cmp_lg_u64 %[tany], 0\n\t"
            "s_cbranch_scc0 4f\n\t"
            B2_LOAD("t1", "w1") B2_LOAD("t2", "w2") B2_LOAD("t3", "w3")
            "v_mov_b32_e32 %[fma], %[MIR]\n\t"
            "v_mov_b32_e32 %[nfa], %[H]\n\t"
            "s_waitcnt lgkmcnt(4)\n\t"
            "v_xad_u32 %[qa], %[t1a], %[nfa], %[hp]\n\t"
            "v_xad_u32 %[qb], %[t1b], %[nfa], %[hp]\n\t"
            B2_WINDOW("%[fma]", "%[fma]", "%[nfa]", "%[nfa]", "tieda", "tiedb", "tieda", "tiedb", "3f")
            "3:\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            "s_branch 5f\n\t"
            "6:\n\t"  // two columns: every row in range is on its chain
            "v_mov_b32_e32 %[alivea], %[hva]\n\t"
            "v_mov_b32_e32 %[aliveb], %[hvb]\n\t"
            "4:\n\t"
            "v_mov_b32_e32 %[tieda], 0\n\t"
            "v_mov_b32_e32 %[tiedb], 0\n\t"
            "5:"
            : B2_SCRATCH, [fma] "=&v"(fma), [fmb] "=&v"(fmb), [nfa] "=&v"(nfa), [nfb] "=&v"(nfb),
              [alivea] "=&v"(alivea), [aliveb] "=&v"(aliveb), [falla] "=&v"(falla), [fallb] "=&v"(fallb),
              [tieda] "=&v"(tieda), [tiedb] "=&v"(tiedb), [tany] "=&s"(tany)
            : B2_COLS, [hva] "v"(hva), [hvb] "v"(hvb)
            : "scc", "memory");
    } else {
        asm volatile(
            "s_waitcnt lgkmcnt(0)\n\t"
            B2_LOAD("t0", "w0") B2_LOAD("t1", "w1") B2_LOAD("t2", "w2") B2_LOAD("t3", "w3")
            "s_waitcnt lgkmcnt(4)\n\t"
            B2_FIRST_NOTIES
            "s_cmp_lt_i32 %[last], 2\n\t"
            "s_cbranch_scc1 6f\n\t"
            B2_WINDOW("%[fma]", "%[fmb]", "%[nfa]", "%[nfb]", "alivea", "aliveb", "hva", "hvb", "2f")
            "2:\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            "s_branch 5f\n\t"
            "6:\n\t"
            "v_mov_b32_e32 %[alivea], %[hva]\n\t"
            "v_mov_b32_e32 %[aliveb], %[hvb]\n\t"
            "5:"
            : B2_SCRATCH, [fma] "=&v"(fma), [fmb] "=&v"(fmb), [nfa] "=&v"(nfa), [nfb] "=&v"(nfb),
              [alivea] "=&v"(alivea), [aliveb] "=&v"(aliveb), [falla] "=&v"(falla), [fallb] "=&v"(fallb)
            : B2_COLS, [hva] "v"(hva), [hvb] "v"(hvb)
            : "scc", "memory");
        tieda = tiedb = 0;
    }
}

// The >= chain alone on both words (fm = 0, nf = ~0).
template <int BITS, int SH = 9>
__device__ __forceinline__ void by2_pos(uint32_t base, const int32_t (&w)[kWin], int32_t last, uint32_t hva,
                                        uint32_t hvb, uint32_t &alivea, uint32_t &aliveb)
{
    using T = Lanes<BITS>;
    uint32_t t0a, t0b, t1a, t1b, t2a, t2b, t3a, t3b, ad, Da, Db, Ea, Eb, qa, qb;
    uint64_t tmp;
    asm volatile(
        "s_waitcnt lgkmcnt(0)\n\t"
        B2_LOAD("t0", "w0") B2_LOAD("t1", "w1") B2_LOAD("t2", "w2") B2_LOAD("t3", "w3")
        "s_waitcnt lgkmcnt(4)\n\t"
        "v_or_b32_e32 %[Da], %[H], %[t1a]\n\t"
        "v_or_b32_e32 %[Db], %[H], %[t1b]\n\t"
        "v_sub_u32_e32 %[Da], %[Da], %[t0a]\n\t"
        "v_sub_u32_e32 %[Db], %[Db], %[t0b]\n\t"
        "v_and_b32_e32 %[alivea], %[Da], %[hva]\n\t"
        "v_and_b32_e32 %[aliveb], %[Db], %[hvb]\n\t"
        "v_xad_u32 %[qa], %[t1a], -1, %[hp]\n\t"
        "v_xad_u32 %[qb], %[t1b], -1, %[hp]\n\t"
        "s_cmp_lt_i32 %[last], 2\n\t"
        "s_cbranch_scc1 2f\n\t"
        B2_WINDOW("0", "0", "-1", "-1", "alivea", "aliveb", "alivea", "aliveb", "2f")
        "2:\n\t"
        "s_waitcnt lgkmcnt(0)"
        : B2_SCRATCH, [alivea] "=&v"(alivea), [aliveb] "=&v"(aliveb)
        : B2_COLS, [hva] "v"(hva), [hvb] "v"(hvb)
        : "scc", "memory");
}

#undef B2_LOAD
#undef B2_PAIR_LAST
#undef B2_PAIR
#undef B2_EXIT_LAST
#undef B2_EXIT
#undef B2_WINDOW
#undef B2_SCRATCH
#undef B2_COLS
#undef B2_F1
#undef B2_F2
#undef B2_F3
#undef B2_F4
#undef B2_F5
#undef B2_F6
#undef B2_F7
#undef B2_F8
#undef B2_F9
#undef B2_AB
#undef B2_FIRST_TIES
#undef B2_FIRST_NOTIES

// ---------------------------------------------------------------------------
// Four lane words per chunk: byte codes in 1024-row chunks (four 256-row
// groups; a staged column is 1024 bytes, word h at +256 h). All four words'
// chains run in one instruction stream, each operation issued for the four
// words in turn, with the arithmetic and the reference q of the two-word
// sequences; one header, one set of column addresses and one set of exit
// tests serve 1024 rows. These sequences take chunks whose rows are all in
// range and hold no two equal values in a row (the top bits of every part
// start set: Hs); other chunks run the two-word sequences on each pair of
// words.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void by4_neg_full(uint32_t base, const int32_t (&w)[kWin], int32_t last, uint32_t (&alive)[4], uint32_t (&fall)[4])
{
    uint32_t t0a, t0b, t0c, t0d, t1a, t1b, t1c, t1d, ad, Da, Db, Dc, Dd, Ea, Eb, Ec, Ed, qa, qb, qc, qd, fma, fmb, fmc, fmd, nfa, nfb, nfc, nfd;
    uint64_t tmp;
    asm volatile(
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_lshl_add_u32 %[ad], %[w0], 10, %[base]\n\t"
        "ds_read_b32 %[t0a], %[ad]\n\t"
        "ds_read_b32 %[t0b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t0c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t0d], %[ad] offset:768\n\t"
        "v_lshl_add_u32 %[ad], %[w1], 10, %[base]\n\t"
        "ds_read_b32 %[t1a], %[ad]\n\t"
        "ds_read_b32 %[t1b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t1c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t1d], %[ad] offset:768\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_or_b32_e32 %[Da], %[Hs], %[t1a]\n\t"
        "v_or_b32_e32 %[Db], %[Hs], %[t1b]\n\t"
        "v_or_b32_e32 %[Dc], %[Hs], %[t1c]\n\t"
        "v_or_b32_e32 %[Dd], %[Hs], %[t1d]\n\t"
        "v_sub_u32_e32 %[Da], %[Da], %[t0a]\n\t"
        "v_sub_u32_e32 %[Db], %[Db], %[t0b]\n\t"
        "v_sub_u32_e32 %[Dc], %[Dc], %[t0c]\n\t"
        "v_sub_u32_e32 %[Dd], %[Dd], %[t0d]\n\t"
        "v_bfi_b32 %[falla], %[Da], 0, %[Hs]\n\t"
        "v_bfi_b32 %[fallb], %[Db], 0, %[Hs]\n\t"
        "v_bfi_b32 %[fallc], %[Dc], 0, %[Hs]\n\t"
        "v_bfi_b32 %[falld], %[Dd], 0, %[Hs]\n\t"
        "v_lshrrev_b32_e32 %[Ea], 7, %[falla]\n\t"
        "v_lshrrev_b32_e32 %[Eb], 7, %[fallb]\n\t"
        "v_lshrrev_b32_e32 %[Ec], 7, %[fallc]\n\t"
        "v_lshrrev_b32_e32 %[Ed], 7, %[falld]\n\t"
        "v_sub_u32_e32 %[fma], %[falla], %[Ea]\n\t"
        "v_sub_u32_e32 %[fmb], %[fallb], %[Eb]\n\t"
        "v_sub_u32_e32 %[fmc], %[fallc], %[Ec]\n\t"
        "v_sub_u32_e32 %[fmd], %[falld], %[Ed]\n\t"
        "v_not_b32_e32 %[nfa], %[fma]\n\t"
        "v_not_b32_e32 %[nfb], %[fmb]\n\t"
        "v_not_b32_e32 %[nfc], %[fmc]\n\t"
        "v_not_b32_e32 %[nfd], %[fmd]\n\t"
        "v_xad_u32 %[qa], %[t1a], %[nfa], %[hp]\n\t"
        "v_xad_u32 %[qb], %[t1b], %[nfb], %[hp]\n\t"
        "v_xad_u32 %[qc], %[t1c], %[nfc], %[hp]\n\t"
        "v_xad_u32 %[qd], %[t1d], %[nfd], %[hp]\n\t"
        "s_cmp_lt_i32 %[last], 2\n\t"
        "s_cbranch_scc1 6f\n\t"
        "v_lshl_add_u32 %[ad], %[w2], 10, %[base]\n\t"
        "ds_read_b32 %[t0a], %[ad]\n\t"
        "ds_read_b32 %[t0b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t0c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t0d], %[ad] offset:768\n\t"
        "v_lshl_add_u32 %[ad], %[w3], 10, %[base]\n\t"
        "ds_read_b32 %[t1a], %[ad]\n\t"
        "ds_read_b32 %[t1b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t1c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t1d], %[ad] offset:768\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_xad_u32 %[Da], %[t0a], %[fma], %[qa]\n\t"
        "v_xad_u32 %[Db], %[t0b], %[fmb], %[qb]\n\t"
        "v_xad_u32 %[Dc], %[t0c], %[fmc], %[qc]\n\t"
        "v_xad_u32 %[Dd], %[t0d], %[fmd], %[qd]\n\t"
        "v_xad_u32 %[qa], %[t0a], %[nfa], %[hp]\n\t"
        "v_xad_u32 %[qb], %[t0b], %[nfb], %[hp]\n\t"
        "v_xad_u32 %[qc], %[t0c], %[nfc], %[hp]\n\t"
        "v_xad_u32 %[qd], %[t0d], %[nfd], %[hp]\n\t"
        "v_xad_u32 %[Ea], %[t1a], %[fma], %[qa]\n\t"
        "v_xad_u32 %[Eb], %[t1b], %[fmb], %[qb]\n\t"
        "v_xad_u32 %[Ec], %[t1c], %[fmc], %[qc]\n\t"
        "v_xad_u32 %[Ed], %[t1d], %[fmd], %[qd]\n\t"
        "v_xad_u32 %[qa], %[t1a], %[nfa], %[hp]\n\t"
        "v_xad_u32 %[qb], %[t1b], %[nfb], %[hp]\n\t"
        "v_xad_u32 %[qc], %[t1c], %[nfc], %[hp]\n\t"
        "v_xad_u32 %[qd], %[t1d], %[nfd], %[hp]\n\t"
        "v_bitop3_b32 %[alivea], %[Hs], %[Da], %[Ea] bitop3:0x80\n\t"
        "v_bitop3_b32 %[aliveb], %[Hs], %[Db], %[Eb] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alivec], %[Hs], %[Dc], %[Ec] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alived], %[Hs], %[Dd], %[Ed] bitop3:0x80\n\t"
        "s_cmp_le_i32 %[last], 3\n\t"
        "s_cbranch_scc1 2f\n\t"
        "v_lshl_add_u32 %[ad], %[w4], 10, %[base]\n\t"
        "ds_read_b32 %[t0a], %[ad]\n\t"
        "ds_read_b32 %[t0b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t0c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t0d], %[ad] offset:768\n\t"
        "v_lshl_add_u32 %[ad], %[w5], 10, %[base]\n\t"
        "ds_read_b32 %[t1a], %[ad]\n\t"
        "ds_read_b32 %[t1b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t1c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t1d], %[ad] offset:768\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_xad_u32 %[Da], %[t0a], %[fma], %[qa]\n\t"
        "v_xad_u32 %[Db], %[t0b], %[fmb], %[qb]\n\t"
        "v_xad_u32 %[Dc], %[t0c], %[fmc], %[qc]\n\t"
        "v_xad_u32 %[Dd], %[t0d], %[fmd], %[qd]\n\t"
        "v_xad_u32 %[qa], %[t0a], %[nfa], %[hp]\n\t"
        "v_xad_u32 %[qb], %[t0b], %[nfb], %[hp]\n\t"
        "v_xad_u32 %[qc], %[t0c], %[nfc], %[hp]\n\t"
        "v_xad_u32 %[qd], %[t0d], %[nfd], %[hp]\n\t"
        "v_xad_u32 %[Ea], %[t1a], %[fma], %[qa]\n\t"
        "v_xad_u32 %[Eb], %[t1b], %[fmb], %[qb]\n\t"
        "v_xad_u32 %[Ec], %[t1c], %[fmc], %[qc]\n\t"
        "v_xad_u32 %[Ed], %[t1d], %[fmd], %[qd]\n\t"
        "v_xad_u32 %[qa], %[t1a], %[nfa], %[hp]\n\t"
        "v_xad_u32 %[qb], %[t1b], %[nfb], %[hp]\n\t"
        "v_xad_u32 %[qc], %[t1c], %[nfc], %[hp]\n\t"
        "v_xad_u32 %[qd], %[t1d], %[nfd], %[hp]\n\t"
        "v_bitop3_b32 %[alivea], %[alivea], %[Da], %[Ea] bitop3:0x80\n\t"
        "v_bitop3_b32 %[aliveb], %[aliveb], %[Db], %[Eb] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alivec], %[alivec], %[Dc], %[Ec] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alived], %[alived], %[Dd], %[Ed] bitop3:0x80\n\t"
        "v_or3_b32 %[Da], %[alivea], %[aliveb], %[alivec]\n\t"
        "v_or_b32_e32 %[Da], %[Da], %[alived]\n\t"
        "v_cmp_ne_u32_e64 %[tmp], 0, %[Da]\n\t"
        "s_cmp_lg_u64 %[tmp], 0\n\t"
        "s_cbranch_scc0 2f\n\t"
        "s_cmp_le_i32 %[last], 5\n\t"
        "s_cbranch_scc1 2f\n\t"
        "v_lshl_add_u32 %[ad], %[w6], 10, %[base]\n\t"
        "ds_read_b32 %[t0a], %[ad]\n\t"
        "ds_read_b32 %[t0b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t0c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t0d], %[ad] offset:768\n\t"
        "v_lshl_add_u32 %[ad], %[w7], 10, %[base]\n\t"
        "ds_read_b32 %[t1a], %[ad]\n\t"
        "ds_read_b32 %[t1b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t1c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t1d], %[ad] offset:768\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_xad_u32 %[Da], %[t0a], %[fma], %[qa]\n\t"
        "v_xad_u32 %[Db], %[t0b], %[fmb], %[qb]\n\t"
        "v_xad_u32 %[Dc], %[t0c], %[fmc], %[qc]\n\t"
        "v_xad_u32 %[Dd], %[t0d], %[fmd], %[qd]\n\t"
        "v_xad_u32 %[qa], %[t0a], %[nfa], %[hp]\n\t"
        "v_xad_u32 %[qb], %[t0b], %[nfb], %[hp]\n\t"
        "v_xad_u32 %[qc], %[t0c], %[nfc], %[hp]\n\t"
        "v_xad_u32 %[qd], %[t0d], %[nfd], %[hp]\n\t"
        "v_xad_u32 %[Ea], %[t1a], %[fma], %[qa]\n\t"
        "v_xad_u32 %[Eb], %[t1b], %[fmb], %[qb]\n\t"
        "v_xad_u32 %[Ec], %[t1c], %[fmc], %[qc]\n\t"
        "v_xad_u32 %[Ed], %[t1d], %[fmd], %[qd]\n\t"
        "v_bitop3_b32 %[alivea], %[alivea], %[Da], %[Ea] bitop3:0x80\n\t"
        "v_bitop3_b32 %[aliveb], %[aliveb], %[Db], %[Eb] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alivec], %[alivec], %[Dc], %[Ec] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alived], %[alived], %[Dd], %[Ed] bitop3:0x80\n\t"
        "2:\n\t"
        "s_branch 5f\n\t"
        "6:\n\t"
        "v_mov_b32_e32 %[alivea], %[Hs]\n\t"
        "v_mov_b32_e32 %[aliveb], %[Hs]\n\t"
        "v_mov_b32_e32 %[alivec], %[Hs]\n\t"
        "v_mov_b32_e32 %[alived], %[Hs]\n\t"
        "5:"
        : [t0a] "=&v"(t0a),
          [t0b] "=&v"(t0b),
          [t0c] "=&v"(t0c),
          [t0d] "=&v"(t0d),
          [t1a] "=&v"(t1a),
          [t1b] "=&v"(t1b),
          [t1c] "=&v"(t1c),
          [t1d] "=&v"(t1d),
          [ad] "=&v"(ad),
          [Da] "=&v"(Da),
          [Db] "=&v"(Db),
          [Dc] "=&v"(Dc),
          [Dd] "=&v"(Dd),
          [Ea] "=&v"(Ea),
          [Eb] "=&v"(Eb),
          [Ec] "=&v"(Ec),
          [Ed] "=&v"(Ed),
          [qa] "=&v"(qa),
          [qb] "=&v"(qb),
          [qc] "=&v"(qc),
          [qd] "=&v"(qd),
          [fma] "=&v"(fma),
          [fmb] "=&v"(fmb),
          [fmc] "=&v"(fmc),
          [fmd] "=&v"(fmd),
          [nfa] "=&v"(nfa),
          [nfb] "=&v"(nfb),
          [nfc] "=&v"(nfc),
          [nfd] "=&v"(nfd),
          [falla] "=&v"(fall[0]),
          [fallb] "=&v"(fall[1]),
          [fallc] "=&v"(fall[2]),
          [falld] "=&v"(fall[3]),
          [alivea] "=&v"(alive[0]),
          [aliveb] "=&v"(alive[1]),
          [alivec] "=&v"(alive[2]),
          [alived] "=&v"(alive[3]),
          [tmp] "=&s"(tmp)
        : [base] "v"(base), [w0] "s"(w[0]), [w1] "s"(w[1]), [w2] "s"(w[2]), [w3] "s"(w[3]), [w4] "s"(w[4]), [w5] "s"(w[5]), [w6] "s"(w[6]), [w7] "s"(w[7]), [last] "s"(last), [Hs] "s"(0x80808080u), [hp] "s"(0x80808081u)
        : "scc", "memory");
}

__device__ __forceinline__ void by4_pos_full(uint32_t base, const int32_t (&w)[kWin], int32_t last, uint32_t (&alive)[4])
{
    uint32_t t0a, t0b, t0c, t0d, t1a, t1b, t1c, t1d, ad, Da, Db, Dc, Dd, Ea, Eb, Ec, Ed, qa, qb, qc, qd;
    uint64_t tmp;
    asm volatile(
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_lshl_add_u32 %[ad], %[w0], 10, %[base]\n\t"
        "ds_read_b32 %[t0a], %[ad]\n\t"
        "ds_read_b32 %[t0b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t0c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t0d], %[ad] offset:768\n\t"
        "v_lshl_add_u32 %[ad], %[w1], 10, %[base]\n\t"
        "ds_read_b32 %[t1a], %[ad]\n\t"
        "ds_read_b32 %[t1b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t1c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t1d], %[ad] offset:768\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_or_b32_e32 %[Da], %[Hs], %[t1a]\n\t"
        "v_or_b32_e32 %[Db], %[Hs], %[t1b]\n\t"
        "v_or_b32_e32 %[Dc], %[Hs], %[t1c]\n\t"
        "v_or_b32_e32 %[Dd], %[Hs], %[t1d]\n\t"
        "v_sub_u32_e32 %[Da], %[Da], %[t0a]\n\t"
        "v_sub_u32_e32 %[Db], %[Db], %[t0b]\n\t"
        "v_sub_u32_e32 %[Dc], %[Dc], %[t0c]\n\t"
        "v_sub_u32_e32 %[Dd], %[Dd], %[t0d]\n\t"
        "v_and_b32_e32 %[alivea], %[Hs], %[Da]\n\t"
        "v_and_b32_e32 %[aliveb], %[Hs], %[Db]\n\t"
        "v_and_b32_e32 %[alivec], %[Hs], %[Dc]\n\t"
        "v_and_b32_e32 %[alived], %[Hs], %[Dd]\n\t"
        "v_xad_u32 %[qa], %[t1a], -1, %[hp]\n\t"
        "v_xad_u32 %[qb], %[t1b], -1, %[hp]\n\t"
        "v_xad_u32 %[qc], %[t1c], -1, %[hp]\n\t"
        "v_xad_u32 %[qd], %[t1d], -1, %[hp]\n\t"
        "s_cmp_lt_i32 %[last], 2\n\t"
        "s_cbranch_scc1 6f\n\t"
        "v_lshl_add_u32 %[ad], %[w2], 10, %[base]\n\t"
        "ds_read_b32 %[t0a], %[ad]\n\t"
        "ds_read_b32 %[t0b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t0c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t0d], %[ad] offset:768\n\t"
        "v_lshl_add_u32 %[ad], %[w3], 10, %[base]\n\t"
        "ds_read_b32 %[t1a], %[ad]\n\t"
        "ds_read_b32 %[t1b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t1c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t1d], %[ad] offset:768\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_xad_u32 %[Da], %[t0a], 0, %[qa]\n\t"
        "v_xad_u32 %[Db], %[t0b], 0, %[qb]\n\t"
        "v_xad_u32 %[Dc], %[t0c], 0, %[qc]\n\t"
        "v_xad_u32 %[Dd], %[t0d], 0, %[qd]\n\t"
        "v_xad_u32 %[qa], %[t0a], -1, %[hp]\n\t"
        "v_xad_u32 %[qb], %[t0b], -1, %[hp]\n\t"
        "v_xad_u32 %[qc], %[t0c], -1, %[hp]\n\t"
        "v_xad_u32 %[qd], %[t0d], -1, %[hp]\n\t"
        "v_xad_u32 %[Ea], %[t1a], 0, %[qa]\n\t"
        "v_xad_u32 %[Eb], %[t1b], 0, %[qb]\n\t"
        "v_xad_u32 %[Ec], %[t1c], 0, %[qc]\n\t"
        "v_xad_u32 %[Ed], %[t1d], 0, %[qd]\n\t"
        "v_xad_u32 %[qa], %[t1a], -1, %[hp]\n\t"
        "v_xad_u32 %[qb], %[t1b], -1, %[hp]\n\t"
        "v_xad_u32 %[qc], %[t1c], -1, %[hp]\n\t"
        "v_xad_u32 %[qd], %[t1d], -1, %[hp]\n\t"
        "v_bitop3_b32 %[alivea], %[alivea], %[Da], %[Ea] bitop3:0x80\n\t"
        "v_bitop3_b32 %[aliveb], %[aliveb], %[Db], %[Eb] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alivec], %[alivec], %[Dc], %[Ec] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alived], %[alived], %[Dd], %[Ed] bitop3:0x80\n\t"
        "s_cmp_le_i32 %[last], 3\n\t"
        "s_cbranch_scc1 2f\n\t"
        "v_lshl_add_u32 %[ad], %[w4], 10, %[base]\n\t"
        "ds_read_b32 %[t0a], %[ad]\n\t"
        "ds_read_b32 %[t0b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t0c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t0d], %[ad] offset:768\n\t"
        "v_lshl_add_u32 %[ad], %[w5], 10, %[base]\n\t"
        "ds_read_b32 %[t1a], %[ad]\n\t"
        "ds_read_b32 %[t1b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t1c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t1d], %[ad] offset:768\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_xad_u32 %[Da], %[t0a], 0, %[qa]\n\t"
        "v_xad_u32 %[Db], %[t0b], 0, %[qb]\n\t"
        "v_xad_u32 %[Dc], %[t0c], 0, %[qc]\n\t"
        "v_xad_u32 %[Dd], %[t0d], 0, %[qd]\n\t"
        "v_xad_u32 %[qa], %[t0a], -1, %[hp]\n\t"
        "v_xad_u32 %[qb], %[t0b], -1, %[hp]\n\t"
        "v_xad_u32 %[qc], %[t0c], -1, %[hp]\n\t"
        "v_xad_u32 %[qd], %[t0d], -1, %[hp]\n\t"
        "v_xad_u32 %[Ea], %[t1a], 0, %[qa]\n\t"
        "v_xad_u32 %[Eb], %[t1b], 0, %[qb]\n\t"
        "v_xad_u32 %[Ec], %[t1c], 0, %[qc]\n\t"
        "v_xad_u32 %[Ed], %[t1d], 0, %[qd]\n\t"
        "v_xad_u32 %[qa], %[t1a], -1, %[hp]\n\t"
        "v_xad_u32 %[qb], %[t1b], -1, %[hp]\n\t"
        "v_xad_u32 %[qc], %[t1c], -1, %[hp]\n\t"
        "v_xad_u32 %[qd], %[t1d], -1, %[hp]\n\t"
        "v_bitop3_b32 %[alivea], %[alivea], %[Da], %[Ea] bitop3:0x80\n\t"
        "v_bitop3_b32 %[aliveb], %[aliveb], %[Db], %[Eb] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alivec], %[alivec], %[Dc], %[Ec] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alived], %[alived], %[Dd], %[Ed] bitop3:0x80\n\t"
        "v_or3_b32 %[Da], %[alivea], %[aliveb], %[alivec]\n\t"
        "v_or_b32_e32 %[Da], %[Da], %[alived]\n\t"
        "v_cmp_ne_u32_e64 %[tmp], 0, %[Da]\n\t"
        "s_cmp_lg_u64 %[tmp], 0\n\t"
        "s_cbranch_scc0 2f\n\t"
        "s_cmp_le_i32 %[last], 5\n\t"
        "s_cbranch_scc1 2f\n\t"
        "v_lshl_add_u32 %[ad], %[w6], 10, %[base]\n\t"
        "ds_read_b32 %[t0a], %[ad]\n\t"
        "ds_read_b32 %[t0b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t0c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t0d], %[ad] offset:768\n\t"
        "v_lshl_add_u32 %[ad], %[w7], 10, %[base]\n\t"
        "ds_read_b32 %[t1a], %[ad]\n\t"
        "ds_read_b32 %[t1b], %[ad] offset:256\n\t"
        "ds_read_b32 %[t1c], %[ad] offset:512\n\t"
        "ds_read_b32 %[t1d], %[ad] offset:768\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_xad_u32 %[Da], %[t0a], 0, %[qa]\n\t"
        "v_xad_u32 %[Db], %[t0b], 0, %[qb]\n\t"
        "v_xad_u32 %[Dc], %[t0c], 0, %[qc]\n\t"
        "v_xad_u32 %[Dd], %[t0d], 0, %[qd]\n\t"
        "v_xad_u32 %[qa], %[t0a], -1, %[hp]\n\t"
        "v_xad_u32 %[qb], %[t0b], -1, %[hp]\n\t"
        "v_xad_u32 %[qc], %[t0c], -1, %[hp]\n\t"
        "v_xad_u32 %[qd], %[t0d], -1, %[hp]\n\t"
        "v_xad_u32 %[Ea], %[t1a], 0, %[qa]\n\t"
        "v_xad_u32 %[Eb], %[t1b], 0, %[qb]\n\t"
        "v_xad_u32 %[Ec], %[t1c], 0, %[qc]\n\t"
        "v_xad_u32 %[Ed], %[t1d], 0, %[qd]\n\t"
        "v_bitop3_b32 %[alivea], %[alivea], %[Da], %[Ea] bitop3:0x80\n\t"
        "v_bitop3_b32 %[aliveb], %[aliveb], %[Db], %[Eb] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alivec], %[alivec], %[Dc], %[Ec] bitop3:0x80\n\t"
        "v_bitop3_b32 %[alived], %[alived], %[Dd], %[Ed] bitop3:0x80\n\t"
        "2:\n\t"
        "s_branch 5f\n\t"
        "6:\n\t"
        "5:"
        : [t0a] "=&v"(t0a),
          [t0b] "=&v"(t0b),
          [t0c] "=&v"(t0c),
          [t0d] "=&v"(t0d),
          [t1a] "=&v"(t1a),
          [t1b] "=&v"(t1b),
          [t1c] "=&v"(t1c),
          [t1d] "=&v"(t1d),
          [ad] "=&v"(ad),
          [Da] "=&v"(Da),
          [Db] "=&v"(Db),
          [Dc] "=&v"(Dc),
          [Dd] "=&v"(Dd),
          [Ea] "=&v"(Ea),
          [Eb] "=&v"(Eb),
          [Ec] "=&v"(Ec),
          [Ed] "=&v"(Ed),
          [qa] "=&v"(qa),
          [qb] "=&v"(qb),
          [qc] "=&v"(qc),
          [qd] "=&v"(qd),
          [alivea] "=&v"(alive[0]),
          [aliveb] "=&v"(alive[1]),
          [alivec] "=&v"(alive[2]),
          [alived] "=&v"(alive[3]),
          [tmp] "=&s"(tmp)
        : [base] "v"(base), [w0] "s"(w[0]), [w1] "s"(w[1]), [w2] "s"(w[2]), [w3] "s"(w[3]), [w4] "s"(w[4]), [w5] "s"(w[5]), [w6] "s"(w[6]), [w7] "s"(w[7]), [last] "s"(last), [Hs] "s"(0x80808080u), [hp] "s"(0x80808081u)
        : "scc", "memory");
}


// Wave-wide masks of the four sub-tiles: bit l of m[b] is bit 7 of byte b
// of lane l's word (one SDWA compare per byte). The trailing wait states
// let any following VALU read the masks.
__device__ __forceinline__ void byte_masks4(uint32_t x, uint64_t &m0, uint64_t &m1, uint64_t &m2, uint64_t &m3)
{
    asm volatile(
        "v_cmp_ne_u32_sdwa %[m0], %[x], 0 src0_sel:BYTE_0 src1_sel:DWORD\n\t"
        "v_cmp_ne_u32_sdwa %[m1], %[x], 0 src0_sel:BYTE_1 src1_sel:DWORD\n\t"
        "v_cmp_ne_u32_sdwa %[m2], %[x], 0 src0_sel:BYTE_2 src1_sel:DWORD\n\t"
        "v_cmp_ne_u32_sdwa %[m3], %[x], 0 src0_sel:BYTE_3 src1_sel:DWORD\n\t"
        "s_nop 1"
        : [m0] "=s"(m0), [m1] "=s"(m1), [m2] "=s"(m2), [m3] "=s"(m3)
        : [x] "v"(x));
}

// Wave-wide masks of the two 64-row sub-tiles of a word of 16-bit parts.
__device__ __forceinline__ void half_masks2(uint32_t x, uint64_t &m0, uint64_t &m1)
{
    asm volatile(
        "v_cmp_ne_u32_sdwa %[m0], %[x], 0 src0_sel:WORD_0 src1_sel:DWORD\n\t"
        "v_cmp_ne_u32_sdwa %[m1], %[x], 0 src0_sel:WORD_1 src1_sel:DWORD\n\t"
        "s_nop 1"
        : [m0] "=s"(m0), [m1] "=s"(m1)
        : [x] "v"(x));
}

// Wave-wide masks of the three 64-row sub-tiles of a word of 10-bit parts:
// x holds only the parts' top bits (9, 19, 29), which lie alone in bytes
// 1, 2 and 3.
__device__ __forceinline__ void t10_masks3(uint32_t x, uint64_t &m0, uint64_t &m1, uint64_t &m2)
{
    asm volatile(
        "v_cmp_ne_u32_sdwa %[m0], %[x], 0 src0_sel:BYTE_1 src1_sel:DWORD\n\t"
        "v_cmp_ne_u32_sdwa %[m1], %[x], 0 src0_sel:BYTE_2 src1_sel:DWORD\n\t"
        "v_cmp_ne_u32_sdwa %[m2], %[x], 0 src0_sel:BYTE_3 src1_sel:DWORD\n\t"
        "s_nop 1"
        : [m0] "=s"(m0), [m1] "=s"(m1), [m2] "=s"(m2)
        : [x] "v"(x));
}

// The sub-tile masks of a word (BITS-bit parts; the top bit of each part).
template <int BITS>
__device__ __forceinline__ void lane_masks(uint32_t x, uint64_t *m)
{
    if constexpr (BITS == 8) byte_masks4(x, m[0], m[1], m[2], m[3]);
    else if constexpr (BITS == 10) t10_masks3(x, m[0], m[1], m[2]);
    else half_masks2(x, m[0], m[1]);
}

// The number of set top bits of all parts of x over the wave: each part's
// mask is counted as soon as it is made, so two scalar pairs hold all of
// them (the SALU reads of a mask the VALU wrote are interlocked).
template <int BITS>
__device__ __forceinline__ int32_t lane_popc(uint32_t x)
{
    uint64_t a, b;
    int32_t c, d;
    if constexpr (BITS == 8) {
        asm volatile(
            "v_cmp_ne_u32_sdwa %[a], %[x], 0 src0_sel:BYTE_0 src1_sel:DWORD\n\t"
            "v_cmp_ne_u32_sdwa %[b], %[x], 0 src0_sel:BYTE_1 src1_sel:DWORD\n\t"
            "s_bcnt1_i32_b64 %[c], %[a]\n\t"
            "v_cmp_ne_u32_sdwa %[a], %[x], 0 src0_sel:BYTE_2 src1_sel:DWORD\n\t"
            "s_bcnt1_i32_b64 %[d], %[b]\n\t"
            "s_add_u32 %[c], %[c], %[d]\n\t"
            "v_cmp_ne_u32_sdwa %[b], %[x], 0 src0_sel:BYTE_3 src1_sel:DWORD\n\t"
            "s_bcnt1_i32_b64 %[d], %[a]\n\t"
            "s_add_u32 %[c], %[c], %[d]\n\t"
            "s_bcnt1_i32_b64 %[d], %[b]\n\t"
            "s_add_u32 %[c], %[c], %[d]"
            : [a] "=&s"(a), [b] "=&s"(b), [c] "=&s"(c), [d] "=&s"(d)
            : [x] "v"(x)
            : "scc");
    } else if constexpr (BITS == 10) {
        asm volatile(
            "v_cmp_ne_u32_sdwa %[a], %[x], 0 src0_sel:BYTE_1 src1_sel:DWORD\n\t"
            "v_cmp_ne_u32_sdwa %[b], %[x], 0 src0_sel:BYTE_2 src1_sel:DWORD\n\t"
            "s_bcnt1_i32_b64 %[c], %[a]\n\t"
            "v_cmp_ne_u32_sdwa %[a], %[x], 0 src0_sel:BYTE_3 src1_sel:DWORD\n\t"
            "s_bcnt1_i32_b64 %[d], %[b]\n\t"
            "s_add_u32 %[c], %[c], %[d]\n\t"
            "s_bcnt1_i32_b64 %[d], %[a]\n\t"
            "s_add_u32 %[c], %[c], %[d]"
            : [a] "=&s"(a), [b] "=&s"(b), [c] "=&s"(c), [d] "=&s"(d)
            : [x] "v"(x)
            : "scc");
    } else {
        asm volatile(
            "v_cmp_ne_u32_sdwa %[a], %[x], 0 src0_sel:WORD_0 src1_sel:DWORD\n\t"
            "v_cmp_ne_u32_sdwa %[b], %[x], 0 src0_sel:WORD_1 src1_sel:DWORD\n\t"
            "s_bcnt1_i32_b64 %[c], %[a]\n\t"
            "s_bcnt1_i32_b64 %[d], %[b]\n\t"
            "s_add_u32 %[c], %[c], %[d]"
            : [a] "=&s"(a), [b] "=&s"(b), [c] "=&s"(c), [d] "=&s"(d)
            : [x] "v"(x)
            : "scc");
    }
    return c;
}

// Plain-code twin of the window (the measurement variant): the same exit
// points; counts one step per 64-row sub-tile (NP per word) and column.
template <int SH, bool COUNT, int NP = 4>
__device__ __forceinline__ void by_window_ref(const unsigned char *__restrict__ base, const int32_t (&w)[kWin],
                                              int32_t last, uint32_t fH, uint32_t nf, uint32_t nx,
                                              uint32_t &alive, uint64_t &steps)
{
#pragma unroll
    for (int u = 2; u < kWin; ++u) {
        const uint32_t t = *reinterpret_cast<const uint32_t *>(base + (w[u] << SH));
        alive &= (t ^ fH) + nx;
        nx = (t ^ nf) + 1u;
        if (COUNT) steps += NP;
        if (u == 3 && last <= 3) return;
        if (u == 5 && (__ballot(alive != 0) == 0 || last <= 5)) return;
    }
}

// Columns kWin..last (long individuals), while any row is left; nx is -x
// of window column 7 (with a row left, the window ran through column 7).
template <int SH, bool COUNT, int NP = 4>
__device__ __forceinline__ void by_tail(const unsigned char *__restrict__ base, const int32_t *__restrict__ c,
                                        const int32_t (&w)[kWin], int32_t last, uint32_t fH, uint32_t nf,
                                        uint32_t &alive, uint64_t &steps)
{
    if (__ballot(alive != 0) == 0) return;
    uint32_t nx = (*reinterpret_cast<const uint32_t *>(base + (w[kWin - 1] << SH)) ^ nf) + 1u;
    for (int32_t u = kWin; u <= last; ++u) {
        if (u > kWin && __ballot(alive != 0) == 0) return;
        const uint32_t t = *reinterpret_cast<const uint32_t *>(base + (c[u] << SH));
        alive &= (t ^ fH) + nx;
        nx = (t ^ nf) + 1u;
        if (COUNT) steps += NP;
    }
}

// One individual on one lane word of SWAR rank codes per row group: four
// 64-row sub-tiles of byte codes (BITS = 8) or two of 16-bit codes
// (BITS = 16). `hv` holds the top bit of the parts whose rows are inside
// the item and the matrix. The codes have no missing value (exclude mode
// uses them only on a matrix without missing cells; include mode's codes
// encode the fill). Sets mw (the top bits of the matching rows' parts) and
// gw (those that match on their negative trend); returns false, leaving
// them unset, when no row matches.
template <int SH, bool NEG, bool COUNT, int BITS = 8, bool TIES = true>
__device__ __forceinline__ bool eval_bytes(const unsigned char *__restrict__ tile, int32_t last,
                                           const int32_t *__restrict__ colidx,
                                           const int32_t *__restrict__ hbegin, const int4 &w03, const int4 &w47,
                                           int lane, uint32_t hv, uint32_t &mw, uint32_t &gw, uint64_t &steps)
{
    using T = Lanes<BITS>;
    constexpr int NP = T::PARTS;
    const unsigned char *base = tile + 4 * lane;
    const int32_t w[kWin] = {w03.x, w03.y, w03.z, w03.w, w47.x, w47.y, w47.z, w47.w};
    auto rd = [&](int32_t col) { return *reinterpret_cast<const uint32_t *>(base + (col << SH)); };
    if (last == 0) {  // one column: every row in range counts
        mw = hv;
        gw = 0;
        if (COUNT) steps += NP;
        return true;
    }
    uint32_t alive, fall = 0, tied = 0;
    if constexpr (COUNT) {
        const uint32_t t0 = rd(w[0]), t1 = rd(w[1]);
        const uint32_t D = (t1 | T::H) - t0, E = (t0 | T::H) - t1;
        uint32_t fH = T::H, nf = ~0u;
        alive = D & hv;
        if constexpr (NEG) {
            tied = D & E & hv;
            fall = E & ~D & hv;
            const uint32_t fm = fall - (fall >> T::SHF);
            fH = fm | T::H;
            nf = ~fm;
            alive = hv;
        }
        steps += NP;
        if (last >= 2) by_window_ref<SH, COUNT, NP>(base, w, last, fH, nf, (t1 ^ nf) + 1u, alive, steps);
        if (NEG && last >= 2 && __ballot(tied != 0) != 0) {
            steps += NP;
            by_window_ref<SH, COUNT, NP>(base, w, last, ~0u, T::H, (t1 ^ T::H) + 1u, tied, steps);
        } else {
            tied = 0;
        }
    } else {
        const uint32_t b = lds_addr(base);
        if constexpr (NEG) by_neg<SH, BITS, TIES>(b, w, last, hv, alive, fall, tied);
        else by_pos<SH, BITS>(b, w, last, hv, alive);
    }
    // No row left on either chain: nothing matches, and the columns past the
    // window (rarely reached: few rows survive eight columns) are skipped.
    if (__ballot((alive | tied) != 0) == 0) return false;
    if (last >= kWin) {
        // The columns past the window (the CSR start is read only here).
        const int32_t *c = colidx + *hbegin;
        if constexpr (NEG) {
            const uint32_t fm = fall - (fall >> T::SHF);
            by_tail<SH, COUNT, NP>(base, c, w, last, fm | T::H, ~fm, alive, steps);
            by_tail<SH, COUNT, NP>(base, c, w, last, ~0u, T::H, tied, steps);
        } else {
            by_tail<SH, COUNT, NP>(base, c, w, last, T::H, ~0u, alive, steps);
        }
        if (__ballot((alive | tied) != 0) == 0) return false;
    }
    mw = alive | tied;
    gw = NEG ? (alive & fall) | (tied & ~alive) : 0u;
    return true;
}

// Plain-code twin of the two-word window (the measurement variant): both
// words in lockstep with the same exits; one step per 64-row sub-tile and
// column.
template <int BITS, bool COUNT, int SH = 9>
__device__ __forceinline__ void by2_window_ref(const unsigned char *__restrict__ base, const int32_t (&w)[kWin],
                                               int32_t last, const uint32_t (&fH)[2], const uint32_t (&nf)[2],
                                               uint32_t (&nx)[2], uint32_t (&alive)[2], uint64_t &steps)
{
#pragma unroll
    for (int u = 2; u < kWin; ++u) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t t = *reinterpret_cast<const uint32_t *>(base + (w[u] << SH) + 256 * h);
            alive[h] &= (t ^ fH[h]) + nx[h];
            nx[h] = (t ^ nf[h]) + 1u;
        }
        if (COUNT) steps += 2 * Lanes<BITS>::PARTS;
        if (u == 3 && last <= 3) return;
        if (u == 5 && (__ballot((alive[0] | alive[1]) != 0) == 0 || last <= 5)) return;
    }
}

// One individual on a chunk of two lane words per row group (byte codes:
// 512 rows, 8 sub-tiles; 16-bit codes: 256 rows, 4 sub-tiles; a column is
// 512 bytes). hva, hvb: the top bits of the in-range rows of each word.
// Sets, per word, mw (the top bits of the matching rows' parts) and gw
// (those that match on their negative trend); returns false, leaving them
// unset, when no row matches.
template <int BITS, bool NEG, bool COUNT, bool TIES, int SH = 9>
__device__ __forceinline__ bool eval_swar2(const unsigned char *__restrict__ tile, int32_t last,
                                           const int32_t *__restrict__ colidx,
                                           const int32_t *__restrict__ hbegin, const int4 &w03, const int4 &w47,
                                           int lane, uint32_t hva, uint32_t hvb, uint32_t (&mw)[2],
                                           uint32_t (&gw)[2], uint64_t &steps)
{
    using T = Lanes<BITS>;
    constexpr int NP = T::PARTS;
    const unsigned char *base = tile + 4 * lane;
    const int32_t w[kWin] = {w03.x, w03.y, w03.z, w03.w, w47.x, w47.y, w47.z, w47.w};
    auto rd = [&](int32_t col, int h) {
        return *reinterpret_cast<const uint32_t *>(base + (col << SH) + 256 * h);
    };
    if (last == 0) {  // one column: every row in range counts
        mw[0] = hva;
        mw[1] = hvb;
        gw[0] = gw[1] = 0;
        if (COUNT) steps += 2 * NP;
        return true;
    }
    uint32_t alive[2], fall[2] = {0, 0}, tied[2] = {0, 0};
    if constexpr (COUNT) {
        uint32_t fH[2], nf[2], nx[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t hv = h ? hvb : hva;
            const uint32_t t0 = rd(w[0], h), t1 = rd(w[1], h);
            const uint32_t D = (t1 | T::H) - t0, E = (t0 | T::H) - t1;
            fH[h] = T::H;
            nf[h] = ~0u;
            alive[h] = D & hv;
            if constexpr (NEG) {
                tied[h] = D & E & hv;
                fall[h] = E & ~D & hv;
                const uint32_t fm = fall[h] - (fall[h] >> T::SHF);
                fH[h] = fm | T::H;
                nf[h] = ~fm;
                alive[h] = hv;
            }
            nx[h] = (t1 ^ nf[h]) + 1u;
        }
        steps += 2 * NP;
        if (last >= 2) by2_window_ref<BITS, COUNT, SH>(base, w, last, fH, nf, nx, alive, steps);
        if (NEG && last >= 2 && __ballot((tied[0] | tied[1]) != 0) != 0) {
            const uint32_t fH2[2] = {~0u, ~0u}, nf2[2] = {T::H, T::H};
            uint32_t nx2[2] = {(rd(w[1], 0) ^ T::H) + 1u, (rd(w[1], 1) ^ T::H) + 1u};
            steps += 2 * NP;
            by2_window_ref<BITS, COUNT, SH>(base, w, last, fH2, nf2, nx2, tied, steps);
        } else {
            tied[0] = tied[1] = 0;
        }
    } else {
        const uint32_t b = lds_addr(base);
        if constexpr (NEG)
            by2_neg<BITS, TIES, SH>(b, w, last, hva, hvb, alive[0], alive[1], fall[0], fall[1], tied[0], tied[1]);
        else by2_pos<BITS, SH>(b, w, last, hva, hvb, alive[0], alive[1]);
    }
    // No row of either word left on either chain: nothing matches, and the
    // columns past the window (rarely reached: few rows survive eight
    // columns) are skipped.
    if (__ballot((alive[0] | alive[1] | tied[0] | tied[1]) != 0) == 0) return false;
    if (last >= kWin) {
        // The columns past the window (the CSR start is read only here).
        const int32_t *c = colidx + *hbegin;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if constexpr (NEG) {
                const uint32_t fm = fall[h] - (fall[h] >> T::SHF);
                by_tail<SH, COUNT, NP>(base + 256 * h, c, w, last, fm | T::H, ~fm, alive[h], steps);
                by_tail<SH, COUNT, NP>(base + 256 * h, c, w, last, ~0u, T::H, tied[h], steps);
            } else {
                by_tail<SH, COUNT, NP>(base + 256 * h, c, w, last, T::H, ~0u, alive[h], steps);
            }
        }
        if (__ballot((alive[0] | alive[1] | tied[0] | tied[1]) != 0) == 0) return false;
    }
    mw[0] = alive[0] | tied[0];
    mw[1] = alive[1] | tied[1];
#pragma unroll
    for (int h = 0; h < 2; ++h) gw[h] = NEG ? (alive[h] & fall[h]) | (tied[h] & ~alive[h]) : 0u;
    return true;
}

// Plain-code twin of the four-word window (the measurement variant): all
// four words in lockstep with the same exits; one step per 64-row sub-tile
// and column.
template <bool COUNT>
__device__ __forceinline__ void by4_window_ref(const unsigned char *__restrict__ base, const int32_t (&w)[kWin],
                                               int32_t last, const uint32_t (&fH)[4], const uint32_t (&nf)[4],
                                               uint32_t (&nx)[4], uint32_t (&alive)[4], uint64_t &steps)
{
#pragma unroll
    for (int u = 2; u < kWin; ++u) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint32_t t = *reinterpret_cast<const uint32_t *>(base + (w[u] << 10) + 256 * h);
            alive[h] &= (t ^ fH[h]) + nx[h];
            nx[h] = (t ^ nf[h]) + 1u;
        }
        if (COUNT) steps += 16;
        if (u == 3 && last <= 3) return;
        if (u == 5 && (__ballot((alive[0] | alive[1] | alive[2] | alive[3]) != 0) == 0 || last <= 5)) return;
    }
}

// One individual on a chunk of four lane words per row group (byte codes,
// 1024 rows, 16 sub-tiles; a column is 1024 bytes). hv: the top bits of the
// in-range rows of each word; full: every row of the chunk is in range.
// Sets, per word, mw and gw as eval_swar2 does; returns false, leaving them
// unset, when no row matches. Full tie-free chunks run the four-word
// sequences; other chunks run the two-word ones on words (0, 1) and (2, 3).
template <bool NEG, bool COUNT, bool TIES>
__device__ __forceinline__ bool eval_swar4(const unsigned char *__restrict__ tile, int32_t last,
                                           const int32_t *__restrict__ colidx,
                                           const int32_t *__restrict__ hbegin, const int4 &w03, const int4 &w47,
                                           int lane, const uint32_t (&hv)[4], bool full, uint32_t (&mw)[4],
                                           uint32_t (&gw)[4], uint64_t &steps)
{
    using T = Lanes<8>;
    if (last == 0) {  // one column: every row in range counts
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            mw[h] = hv[h];
            gw[h] = 0;
        }
        if (COUNT) steps += 16;
        return true;
    }
    if (!full || (NEG && TIES)) {
        uint32_t m2[2] = {0, 0}, g2[2] = {0, 0}, m3[2] = {0, 0}, g3[2] = {0, 0};
        const bool a = eval_swar2<8, NEG, COUNT, TIES, 10>(tile, last, colidx, hbegin, w03, w47, lane, hv[0], hv[1],
                                                            m2, g2, steps);
        const bool b = eval_swar2<8, NEG, COUNT, TIES, 10>(tile + 512, last, colidx, hbegin, w03, w47, lane, hv[2],
                                                            hv[3], m3, g3, steps);
        if (!a && !b) return false;
        mw[0] = a ? m2[0] : 0u;
        mw[1] = a ? m2[1] : 0u;
        gw[0] = a ? g2[0] : 0u;
        gw[1] = a ? g2[1] : 0u;
        mw[2] = b ? m3[0] : 0u;
        mw[3] = b ? m3[1] : 0u;
        gw[2] = b ? g3[0] : 0u;
        gw[3] = b ? g3[1] : 0u;
        return true;
    }
    const unsigned char *base = tile + 4 * lane;
    const int32_t w[kWin] = {w03.x, w03.y, w03.z, w03.w, w47.x, w47.y, w47.z, w47.w};
    uint32_t alive[4], fall[4] = {0, 0, 0, 0};
    if constexpr (COUNT) {
        uint32_t fH[4], nf[4], nx[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint32_t t0 = *reinterpret_cast<const uint32_t *>(base + (w[0] << 10) + 256 * h);
            const uint32_t t1 = *reinterpret_cast<const uint32_t *>(base + (w[1] << 10) + 256 * h);
            const uint32_t D = (t1 | T::H) - t0;
            fH[h] = T::H;
            nf[h] = ~0u;
            alive[h] = D & T::H;
            if constexpr (NEG) {
                fall[h] = ~D & T::H;
                const uint32_t fm = fall[h] - (fall[h] >> T::SHF);
                fH[h] = fm | T::H;
                nf[h] = ~fm;
                alive[h] = T::H;
            }
            nx[h] = (t1 ^ nf[h]) + 1u;
        }
        steps += 16;
        if (last >= 2) by4_window_ref<COUNT>(base, w, last, fH, nf, nx, alive, steps);
    } else {
        const uint32_t b = lds_addr(base);
        if constexpr (NEG) by4_neg_full(b, w, last, alive, fall);
        else by4_pos_full(b, w, last, alive);
    }
    if (__ballot((alive[0] | alive[1] | alive[2] | alive[3]) != 0) == 0) return false;
    if (last >= kWin) {
        // The columns past the window (the CSR start is read only here).
        const int32_t *c = colidx + *hbegin;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint32_t fm = NEG ? fall[h] - (fall[h] >> T::SHF) : 0u;
            by_tail<10, COUNT, 4>(base + 256 * h, c, w, last, fm | T::H, ~fm, alive[h], steps);
        }
        if (__ballot((alive[0] | alive[1] | alive[2] | alive[3]) != 0) == 0) return false;
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        mw[h] = alive[h];
        gw[h] = NEG ? alive[h] & fall[h] : 0u;
    }
    return true;
}

// One individual read straight from the column-major matrix (matrices too
// wide to stage). `xr` points at row (row0 + lane) of column 0; `sub`
// holds the element offsets of the L sub-tiles (clamped by the caller so
// that every read stays inside the matrix).
template <int L, bool NEG, bool COUNT>
__device__ __forceinline__ void eval_direct(const float *__restrict__ xr, int64_t ld,
                                            const int64_t (&sub)[L], int32_t last,
                                            const int32_t *__restrict__ c, float fill,
                                            bool subst, const uint64_t (&valid)[L],
                                            uint64_t (&M)[L], uint64_t (&G)[L], uint64_t &steps)
{
    auto load = [&](int32_t col, int s) {
        float v = xr[(int64_t)col * ld + sub[s]];
        if (subst) v = v != v ? fill : v;
        return v;
    };
    uint64_t P[L], N[L];
    float prev[L];
#pragma unroll
    for (int s = 0; s < L; ++s) {
        prev[s] = load(c[0], s);
        P[s] = __ballot(prev[s] == prev[s]) & valid[s];
        N[s] = NEG ? P[s] : 0ull;
    }
    if (COUNT) steps += L;
    for (int32_t u = 1; u <= last; u += 2) {
        const int32_t ca = c[u], cb = c[min(u + 1, last)];
        uint64_t x = 0;
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const float va = load(ca, s), vb = load(cb, s);
            P[s] &= __ballot(va >= prev[s]) & __ballot(vb >= va);
            if (NEG) N[s] &= __ballot(va <= prev[s]) & __ballot(vb <= va);
            prev[s] = vb;
            x |= P[s] | N[s];
        }
        if (COUNT) steps += 2 * L;
        if (x == 0) break;
    }
#pragma unroll
    for (int s = 0; s < L; ++s) {
        M[s] = P[s] | N[s];
        G[s] = N[s] & ~P[s];
    }
}

// Store the per-sub-tile words of one individual with one coalesced store:
// lane s writes word s.
template <int L>
__device__ __forceinline__ void store_words(uint64_t *__restrict__ dst, const uint64_t (&w)[L],
                                            int nl, int lane)
{
    uint64_t mine = 0;
#pragma unroll
    for (int s = 0; s < L; ++s)
        if (lane == s) mine = w[s];
    if (lane < nl) dst[lane] = mine;
}

// ---------------------------------------------------------------------------
// The header fields the evaluation uses (length, CSR start, window), read
// with scalar loads and materialised together: one scalar-memory round trip
// instead of a dependent load per field on the early-exit path.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_head(const IndHead *__restrict__ hb, int32_t ii, int4 (&hv)[3])
{
    const int4 *p = reinterpret_cast<const int4 *>(hb + ii);
    hv[0] = p[0];  // k, begin
    hv[1] = p[2];  // win[0..3]
    hv[2] = p[3];  // win[4..7]
    asm volatile("" ::"s"(hv[0].x), "s"(hv[0].y), "s"(hv[1].x), "s"(hv[1].y), "s"(hv[1].z),
                 "s"(hv[1].w), "s"(hv[2].x), "s"(hv[2].y), "s"(hv[2].z), "s"(hv[2].w));
}


// ---------------------------------------------------------------------------
// One work item: individuals [i0, i0 + np) of request d on tiles [t0, t1).
// `tile` and `cnt` are this block's LDS areas; wave w takes the group's
// individuals w, w + W, w + 2W, ... on every chunk, so each count has a
// single writer. Ends with a barrier, so a persistent block can start its
// next item right away.
// ---------------------------------------------------------------------------
// C16: the counts as 16-bit halves of one word per individual (the plain
// kernel with 16-bit codes, whose wide tiles leave little LDS for counts;
// the planner keeps every range of such a launch below 65,536 rows).
template <int L, bool NEG, int STAGE, bool COUNT, bool C16 = false>
__device__ __forceinline__ void run_item(const ReqDesc &d, const IndHead *__restrict__ heads,
                                         int32_t i0, int32_t np, int64_t t0, int64_t t1,
                                         float *tile, int32_t *cnt, uint64_t &steps)
{
    constexpr int T = L * kWave;
    const int lane = threadIdx.x & (kWave - 1);
    // Wave index as a scalar: every per-individual quantity derived from it
    // (lengths, column indices, masks) then lives in scalar registers.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int W = blockDim.x / kWave;
    const int64_t words = (d.rows + 63) / 64;
    const bool include = (d.flags & kFlagInclude) != 0;
    const IndHead *hb = heads + d.head_base + i0;

    constexpr bool c16 = C16;
    for (int32_t t = threadIdx.x; t < (c16 ? np : 2 * np); t += blockDim.x) cnt[t] = 0;

    // Byte or 16-bit codes (SWAR stagings): a chunk holds L * 64 * RB bytes
    // of every column (one or two lane words per row); every thread copies
    // up to two 16-byte pieces of it (piece idx = bytes 16 * (idx % pieces)
    // of column idx / pieces) through registers, and the pieces of the next
    // chunk are loaded while the current one is evaluated. Pieces past
    // 2 * blockDim are copied directly.
    constexpr bool kSwar = STAGE == STAGE_BYTES || STAGE == STAGE_HALVES || STAGE == STAGE_T10;
    constexpr bool kT10 = STAGE == STAGE_T10;
    constexpr int BITS = STAGE == STAGE_HALVES ? 16 : kT10 ? 10 : 8;
    constexpr int PARTS = kT10 ? 3 : 32 / BITS;      // rows (sub-tiles) per lane word
    constexpr int NWORDS = L >= PARTS ? L / PARTS : 1;  // lane words per chunk
    constexpr int CB = 256 * NWORDS;                  // bytes of one column per chunk
    constexpr int PL = NWORDS == 4 ? 6 : NWORDS == 2 ? 5 : 4;  // log2 of the 16-byte pieces per column
    // A chunk starts on a multiple of L tiles: its bytes in a column, and
    // the index of its tie flag (one per 512 rows; 10-bit codes: one per
    // 192-row group, two groups in a chunk of two words).
    // (byte chunks of 16 sub-tiles may start on any multiple of 8 tiles)
    auto chunk_at = [](int64_t tile) { return kT10 ? tile / 3 * 256 : tile * kWave * (BITS / 8); };
    auto tie_at = [](int64_t tile) { return kT10 ? tile / 3 : (tile * kWave) >> 9; };
    const int btotal = kSwar ? d.cols << PL : 0;
    const int idx0 = threadIdx.x, idx1 = threadIdx.x + blockDim.x;
    const uint8_t *src0 = d.B + (int64_t)(idx0 >> PL) * d.ldb + 16 * (idx0 & ((1 << PL) - 1));
    const uint8_t *src1 = d.B + (int64_t)(idx1 >> PL) * d.ldb + 16 * (idx1 & ((1 << PL) - 1));
    uint4 pre0 = {0, 0, 0, 0}, pre1 = {0, 0, 0, 0};
    // Pieces prefetched per thread (four-word chunks keep one, to leave
    // registers to the four words' chains).
    constexpr bool kPre1 = NWORDS != 4;
    // Chunks that span two tie flags: 1024 rows of byte codes, two 192-row
    // groups of 10-bit codes.
    constexpr bool kTwoFlags = NWORDS == 4 || (kT10 && NWORDS == 2);
    int32_t tie_pre = 1;  // the next chunk's tie flag, loaded with its bytes
    if constexpr (kSwar) {
        if (t0 < t1) {
            const int64_t r0 = chunk_at(t0);
            if (idx0 < btotal) pre0 = *reinterpret_cast<const uint4 *>(src0 + r0);
            if (kPre1 && idx1 < btotal) pre1 = *reinterpret_cast<const uint4 *>(src1 + r0);
            tie_pre = d.T[tie_at(t0)];
            if (kTwoFlags) tie_pre |= d.T[tie_at(t0) + 1];  // (two flags per chunk)
        }
    }

    for (int64_t tb = t0; tb < t1; tb += L) {
        const int nl = (int)min<int64_t>(L, t1 - tb);
        const int64_t row0 = tb * kWave;
        uint64_t valid[L];
#pragma unroll
        for (int s = 0; s < L; ++s) valid[s] = __ballot(s < nl && row0 + s * kWave + lane < d.rows);

        __syncthreads();  // counts initialised; the previous chunk's readers are done
        if constexpr (STAGE == STAGE_CODES) {
            // Rows [row0, row0 + nl*64) of every column's rank codes, 4 rows
            // (8 bytes) per thread; codes of include mode already encode the
            // fill value.
            uint16_t *tile16 = reinterpret_cast<uint16_t *>(tile);
            const int q_per_col = nl * (kWave / 4);
            const int total = q_per_col * d.cols;
            for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
                const int c = idx / q_per_col;
                const int q = idx - c * q_per_col;
                *reinterpret_cast<uint2 *>(tile16 + (size_t)c * T + 4 * q) =
                    *reinterpret_cast<const uint2 *>(d.C + (int64_t)c * d.ld + row0 + 4 * q);
            }
            if (nl < L || row0 + T > d.rows) {  // as below: outside rows never match
                __syncthreads();
                const int64_t first = min<int64_t>(d.rows - row0, (int64_t)nl * kWave);
                const int tail = T * d.cols;
                for (int idx = threadIdx.x; idx < tail; idx += blockDim.x) {
                    const int r = idx % T;
                    if (r >= first) tile16[idx] = kCodeNaN;
                }
            }
            __syncthreads();
        }
        // SWAR codes: per lane word, the top bit of each part whose row is
        // in range, and whether a row of the chunk holds two equal values.
        uint32_t hvalid[NWORDS] = {};
        bool ties = true;
        bool full = true;  // every row of the chunk is in range
        if constexpr (kSwar) {
            static_assert(STAGE == STAGE_HALVES ? (L == 2 || L == 4) : kT10 ? (L == 3 || L == 6) : (L == 4 || L == 8 || L == 16),
                          "one, two or four lane words per row of a chunk");
            ties = __builtin_amdgcn_readfirstlane(tie_pre) != 0;  // (uniform: one flag per chunk)
            // The L * 64 rows [row0, row0 + 64 L) of every column, in their
            // interleaved order; rows outside the item or the matrix are
            // left out of `hvalid` instead.
            uint4 *tile4 = reinterpret_cast<uint4 *>(tile);
            if (idx0 < btotal) tile4[idx0] = pre0;
            if (kPre1 && idx1 < btotal) tile4[idx1] = pre1;
            for (int idx = kPre1 ? idx1 + blockDim.x : idx1; idx < btotal; idx += blockDim.x)
                tile4[idx] = *reinterpret_cast<const uint4 *>(d.B + (int64_t)(idx >> PL) * d.ldb + chunk_at(tb) +
                                                              16 * (idx & ((1 << PL) - 1)));
            if (nl == L && row0 + L * kWave <= d.rows) {
#pragma unroll
                for (int h = 0; h < NWORDS; ++h) hvalid[h] = Lanes<BITS>::H;
            } else {
                full = false;
#pragma unroll
                for (int s = 0; s < L; ++s)
                    if (s < nl && row0 + s * kWave + lane < d.rows)
                        hvalid[s / PARTS] |= 1u << (BITS * (s % PARTS) + BITS - 1);
            }
            __syncthreads();
            if (tb + L < t1) {
                const int64_t r1 = chunk_at(tb + L);
                if (idx0 < btotal) pre0 = *reinterpret_cast<const uint4 *>(src0 + r1);
                if (kPre1 && idx1 < btotal) pre1 = *reinterpret_cast<const uint4 *>(src1 + r1);
                tie_pre = d.T[tie_at(tb + L)];
                if (kTwoFlags) tie_pre |= d.T[tie_at(tb + L) + 1];
            }
        }
        if constexpr (STAGE == STAGE_LDS) {
            // Rows [row0, row0 + nl*64) of every column, 4 rows per thread.
            const int q_per_col = nl * (kWave / 4);
            const int total = q_per_col * d.cols;
            const float fill = d.fill;
            for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
                const int c = idx / q_per_col;
                const int q = idx - c * q_per_col;
                float4 v = *reinterpret_cast<const float4 *>(d.X + (int64_t)c * d.ld + row0 + 4 * q);
                if (include) {
                    v.x = v.x != v.x ? fill : v.x;
                    v.y = v.y != v.y ? fill : v.y;
                    v.z = v.z != v.z ? fill : v.z;
                    v.w = v.w != v.w ? fill : v.w;
                }
                *reinterpret_cast<float4 *>(tile + (size_t)c * T + 4 * q) = v;
            }
            if (L >= 2 && (nl < L || row0 + T > d.rows)) {
                // The interleaved evaluation reads all L sub-tiles and takes
                // no row mask: rows outside this item's range or past the end
                // of the matrix hold NaN, so they never match.
                __syncthreads();
                const int64_t first = min<int64_t>(d.rows - row0, (int64_t)nl * kWave);
                const int tail = T * d.cols;
                for (int idx = threadIdx.x; idx < tail; idx += blockDim.x) {
                    const int r = idx % T;
                    if (r >= first) tile[idx] = __builtin_nanf("");
                }
            }
            __syncthreads();
        }

        // The individuals of this wave on the staged chunk.
        auto individuals = [&](auto masks_tag, auto ties_tag) {
        constexpr bool MASKS = decltype(masks_tag)::value;
        constexpr bool TIES = decltype(ties_tag)::value;  // (SWAR chunks only)
        // One individual (header hv) on the staged chunk.
        // Lane 0 adds an individual's two counts to the block's LDS
        // accumulators; no result is returned, so nothing waits for it.
        auto add_counts = [&](int32_t ii, int32_t pm, int32_t pg) {
            if (pm | pg) {
                uint64_t save;
                uint32_t va, vm, vg;
                if constexpr (c16) {
                    const uint32_t a = lds_addr(cnt + ii);
                    const uint32_t both = (uint32_t)pm | ((uint32_t)pg << 16);
                    asm volatile(
                        "s_mov_b64 %[save], exec\n\t"
                        "s_mov_b64 exec, 1\n\t"
                        "v_mov_b32 %[va], %[a]\n\t"
                        "v_mov_b32 %[vm], %[both]\n\t"
                        "ds_add_u32 %[va], %[vm]\n\t"
                        "s_mov_b64 exec, %[save]"
                        : [save] "=&s"(save), [va] "=&v"(va), [vm] "=&v"(vm)
                        : [a] "s"(a), [both] "s"(both)
                        : "memory");
                } else {
                    const uint32_t a = lds_addr(cnt + 2 * ii);
                    asm volatile(
                        "s_mov_b64 %[save], exec\n\t"
                        "s_mov_b64 exec, 1\n\t"
                        "v_mov_b32 %[va], %[a]\n\t"
                        "v_mov_b32 %[vm], %[pm]\n\t"
                        "v_mov_b32 %[vg], %[pg]\n\t"
                        "ds_add_u32 %[va], %[vm]\n\t"
                        "ds_add_u32 %[va], %[vg] offset:4\n\t"
                        "s_mov_b64 exec, %[save]"
                        : [save] "=&s"(save), [va] "=&v"(va), [vm] "=&v"(vm), [vg] "=&v"(vg)
                        : [a] "s"(a), [pm] "s"(pm), [pg] "s"(pg)
                        : "memory");
                }
            }
        };
        auto one = [&](const int4 (&hv)[3], int32_t ii) {
            const int32_t k = hv[0].x;
            if constexpr (kSwar && !MASKS) {
                // Counts only: the match words' parts are counted as they
                // are made (no masks exist on this path).
                if (k == 0) return;
                const auto *tl = reinterpret_cast<const unsigned char *>(tile);
                if constexpr (NWORDS == 4) {
                    if (!full || (NEG && TIES)) {
                        // each pair of words on its own, counted as it ends
                        // (fewer registers live than four words' results)
                        int32_t pm = 0, pg = 0;
#pragma unroll
                        for (int half = 0; half < 2; ++half) {
                            if (8 * half >= nl) break;  // (a half chunk at the end of a range)
                            uint32_t m2[2] = {0, 0}, g2[2] = {0, 0};
                            if (eval_swar2<8, NEG, COUNT, TIES, 10>(tl + 512 * half, k - 1, d.colidx, &hb[ii].begin,
                                                                    hv[1], hv[2], lane, hvalid[2 * half],
                                                                    hvalid[2 * half + 1], m2, g2, steps)) {
#pragma unroll
                                for (int h = 0; h < 2; ++h) {
                                    pm += lane_popc<8>(m2[h]);
                                    if constexpr (NEG) pg += lane_popc<8>(g2[h]);
                                }
                            }
                        }
                        add_counts(ii, pm, pg);
                        return;
                    }
                }
                uint32_t mw[NWORDS] = {}, gw[NWORDS] = {};
                bool any;
                if constexpr (NWORDS == 4)
                    any = eval_swar4<NEG, COUNT, TIES>(tl, k - 1, d.colidx, &hb[ii].begin, hv[1], hv[2], lane,
                                                       hvalid, true, mw, gw, steps);
                else if constexpr (NWORDS == 2)
                    any = eval_swar2<BITS, NEG, COUNT, TIES>(tl, k - 1, d.colidx, &hb[ii].begin, hv[1], hv[2], lane,
                                                             hvalid[0], hvalid[NWORDS - 1], mw, gw, steps);
                else
                    any = eval_bytes<8, NEG, COUNT, BITS, TIES>(tl, k - 1, d.colidx, &hb[ii].begin, hv[1], hv[2],
                                                                lane, hvalid[0], mw[0], gw[0], steps);
                if (!any) return;
                int32_t pm = 0, pg = 0;
#pragma unroll
                for (int h = 0; h < NWORDS; ++h) {
                    pm += lane_popc<BITS>(mw[h]);
                    if constexpr (NEG) pg += lane_popc<BITS>(gw[h]);
                }
                add_counts(ii, pm, pg);
                return;
            }
            uint64_t M[L], G[L];
            if (k == 0) {
#pragma unroll
                for (int s = 0; s < L; ++s) M[s] = G[s] = 0;
            } else {
                bool live = true;  // (byte codes: counted per 256-row group below)
                int32_t pm = 0, pg = 0;
                if constexpr (kSwar) {
                    // One or two lane words per row: the evaluation returns
                    // the words of matching rows; the masks are made only
                    // when they are stored, else each word's parts are
                    // counted directly.
                    live = false;
                    const auto *tl = reinterpret_cast<const unsigned char *>(tile);
                    uint32_t mw[2] = {0, 0}, gw[2] = {0, 0};
                    bool any;
                    if constexpr (NWORDS == 4)
                        any = false;  // (never reached: four-word chunks take the count-only path above)
                    else if constexpr (NWORDS == 2)
                        any = eval_swar2<BITS, NEG, COUNT, TIES>(tl, k - 1, d.colidx, &hb[ii].begin, hv[1], hv[2],
                                                                 lane, hvalid[0], hvalid[NWORDS - 1], mw, gw, steps);
                    else
                        any = eval_bytes<8, NEG, COUNT, BITS, TIES>(tl, k - 1, d.colidx, &hb[ii].begin, hv[1], hv[2],
                                                                    lane, hvalid[0], mw[0], gw[0], steps);
                    if (any) {
#pragma unroll
                        for (int h = 0; h < NWORDS; ++h) {
                            if constexpr (MASKS) {
                                lane_masks<BITS>(mw[h], M + h * PARTS);
                                lane_masks<BITS>(gw[h], G + h * PARTS);
                            } else {
                                pm += lane_popc<BITS>(mw[h]);
                                if constexpr (NEG) pg += lane_popc<BITS>(gw[h]);
                            }
                        }
                        if constexpr (MASKS) {
#pragma unroll
                            for (int s = 0; s < L; ++s) {
                                pm += __popcll(M[s]);
                                pg += __popcll(G[s]);
                            }
                        }
                    } else if constexpr (MASKS) {
#pragma unroll
                        for (int s = 0; s < L; ++s) M[s] = G[s] = 0;
                    }
                } else if constexpr (STAGE == STAGE_CODES) {
                    static_assert(L >= 2, "rank codes are staged for 2 or 4 sub-tiles");
                    const int32_t *c = d.colidx + hv[0].y;
                    eval_lds_il<L, NEG, COUNT, uint16_t>(reinterpret_cast<const unsigned char *>(tile), k - 1,
                                                         c, hv[1], hv[2], lane, M, G, steps);
                } else if constexpr (STAGE == STAGE_LDS) {
                    const int32_t *c = d.colidx + hv[0].y;
                    if constexpr (L >= 2)
                        eval_lds_il<L, NEG, COUNT, float>(reinterpret_cast<const unsigned char *>(tile), k - 1, c,
                                                          hv[1], hv[2], lane, M, G, steps);
                    else
                        eval_lds<L, NEG, COUNT>(reinterpret_cast<const unsigned char *>(tile), k - 1, c,
                                                hv[1], hv[2], lane * 4, valid, M, G, steps);
                } else {
                    // Sub-tiles past the last tile are clamped onto it (their
                    // rows are masked out by `valid`).
                    const int64_t last_row0 = (words - 1) * kWave;
                    int64_t sub[L];
#pragma unroll
                    for (int s = 0; s < L; ++s) sub[s] = min<int64_t>(row0 + s * kWave, last_row0) - row0;
                    const int32_t *c = d.colidx + hv[0].y;
                    eval_direct<L, NEG, COUNT>(d.X + row0 + lane, d.ld, sub, k - 1, c, d.fill,
                                               (d.flags & kFlagSubst) != 0, valid, M, G, steps);
                }
                if (live) {
#pragma unroll
                    for (int s = 0; s < L; ++s) {
                        pm += __popcll(M[s]);
                        pg += __popcll(G[s]);
                    }
                }
                add_counts(ii, pm, pg);
            }
            if constexpr (MASKS) {
                const int64_t i = i0 + ii;
                if (d.mmask) store_words<L>(d.mmask + i * words + tb, M, nl, lane);
                if (d.nmask) store_words<L>(d.nmask + i * words + tb, G, nl, lane);
            }
        };
        for (int32_t ii = wave; ii < np; ii += W) {
            int4 hv[3];
            load_head(hb, ii, hv);
            one(hv, ii);
        }
        };
        // The loop is compiled with and without the mask stores, and for
        // SWAR chunks with and without the tie chain (the chunk's flag,
        // decided once here rather than per individual).
        if constexpr (kSwar && NWORDS == 4) {
            // (counts only: the planner stages four words per row group only
            // for calls without masks, and the launch checks it)
            if (ties) individuals(std::false_type{}, std::true_type{});
            else individuals(std::false_type{}, std::false_type{});
        } else if constexpr (kSwar) {
            if (d.mmask || d.nmask) {
                if (ties) individuals(std::true_type{}, std::true_type{});
                else individuals(std::true_type{}, std::false_type{});
            } else {
                if (ties) individuals(std::false_type{}, std::true_type{});
                else individuals(std::false_type{}, std::false_type{});
            }
        } else {
            if (d.mmask || d.nmask) individuals(std::true_type{}, std::true_type{});
            else individuals(std::false_type{}, std::true_type{});
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the count adds, before the barrier
    }

    __syncthreads();
    for (int32_t t = threadIdx.x; t < np; t += blockDim.x) {
        const int32_t m = c16 ? (int32_t)((uint32_t)cnt[t] & 0xffffu) : cnt[2 * t];
        const int32_t g = c16 ? (int32_t)((uint32_t)cnt[t] >> 16) : cnt[2 * t + 1];
        if (m > 0) atomicAdd(d.matched + i0 + t, m);
        if (g > 0 && d.negative) atomicAdd(d.negative + i0 + t, g);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Plain evaluation: one block per (tile range, individual group).
// ---------------------------------------------------------------------------
template <int L, bool NEG, int STAGE, bool COUNT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
k_eval(ReqDesc d, const IndHead *__restrict__ heads, int32_t P, int32_t n_tiles,
       unsigned long long *step_counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const size_t tb = tile_bytes_of(L, d.cols, STAGE);
    float *tile = reinterpret_cast<float *>(smem);
    int32_t *cnt = reinterpret_cast<int32_t *>(smem + tb);
    // Block (x, y) is tile range x of group y: blocks b and b + 256 (in
    // dispatch order), which share a CU when two are resident, stage the
    // same rows for two groups, and the second finds them in the CU's L1.
    // Byte codes (narrow matrices, small chunks) gain more from header
    // locality: blocks are dispatched round-robin over the 8 XCDs (block b
    // to XCD b mod 8), so with R ranges a multiple of 8, XCD x takes the
    // contiguous ranges [x R/8, (x+1) R/8) for every group (the groups
    // re-reading a range share that XCD's L2) and its k-th block takes group
    // k mod G (the blocks sharing a CU, k and k + 32, mostly share a group,
    // whose headers stay in the scalar cache).
    const uint32_t R = gridDim.x, G = gridDim.y;
    int32_t grp = (int32_t)blockIdx.y, rng = (int32_t)blockIdx.x;
    if (STAGE == STAGE_BYTES && R % 8 == 0) {
        const uint32_t b = blockIdx.y * R + blockIdx.x, k = b / 8;
        grp = (int32_t)(k % G);
        rng = (int32_t)((b % 8) * (R / 8) + k / G);
    }
    const int32_t i0 = grp * P;
    const int32_t np = min(P, d.n - i0);
    if (np <= 0) return;
    // Tile ranges start on a multiple of L, so only the matrix's last chunk
    // can be partial.
    // Ranges start on a multiple of RG tiles: L, except byte codes in chunks
    // of 16 sub-tiles, whose ranges are cut in units of 8 (a range then ends
    // with a half chunk when it holds an odd number of units, so that the
    // ranges stay as even as with 8-sub-tile chunks).
    constexpr int RG = (STAGE == STAGE_BYTES && L == 16) ? 8 : L;
    const int64_t n_chunks = (n_tiles + RG - 1) / RG;
    const int64_t t0 = (int64_t)rng * n_chunks / gridDim.x * RG;
    const int64_t t1 = min<int64_t>(n_tiles, (int64_t)(rng + 1) * n_chunks / gridDim.x * RG);
    uint64_t steps = 0;
    run_item<L, NEG, STAGE, COUNT, STAGE == STAGE_HALVES || STAGE == STAGE_T10>(d, heads, i0, np, t0, t1, tile,
                                                                                 cnt, steps);
    if (COUNT && (threadIdx.x & (kWave - 1)) == 0 && steps)
        atomicAdd(step_counter, (unsigned long long)steps);
}

// ---------------------------------------------------------------------------
// Batched evaluation: persistent blocks take work items from the counter in
// the batch header until none are left; each item carries its request
// (matrix, population, flags, outputs).
// ---------------------------------------------------------------------------
// SET: the stagings this instance handles (kBatchSet* bits): a batch whose
// requests all stage one kind of SWAR codes runs an instance compiled for
// that kind alone, whose registers are not shared with the other paths.
template <int L, int SET, bool COUNT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
k_eval_batch(BatchHeader *hdr, const ReqDesc *__restrict__ descs, const Item *__restrict__ items,
             const IndHead *__restrict__ heads, int32_t tile_bytes, int32_t P,
             unsigned long long *step_counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t s_item;
    float *tile = reinterpret_cast<float *>(smem);
    int32_t *cnt = reinterpret_cast<int32_t *>(smem + tile_bytes);
    (void)P;
    const int32_t n_items = __builtin_amdgcn_readfirstlane(hdr->n_items);
    uint64_t steps = 0;
    while (true) {
        if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(&hdr->counter, 1u);
        __syncthreads();
        const int32_t id = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();  // every wave has read s_item before thread 0 rewrites it
        if (id >= n_items) break;
        const Item it = items[id];
        const ReqDesc d = descs[it.req];
        const bool neg = (d.flags & kFlagNeg) != 0;
        // SWAR codes in batches: one lane word per row group, at the number
        // of sub-tiles of the codes (bytes 4, 10-bit codes 3, 16-bit codes
        // 2; the planner cuts each request's tile ranges to it). The
        // two-word sequences are left to plain launches: beside the other
        // paths of a persistent kernel they would not fit its registers.
        if constexpr ((SET & kBatchSetBytes) != 0) {
            if (d.flags & kFlagBytes) {
                if (neg) run_item<4, true, STAGE_BYTES, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                else run_item<4, false, STAGE_BYTES, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                continue;
            }
        }
        if constexpr ((SET & kBatchSetT10) != 0) {
            if (d.flags & kFlagT10) {
                if (neg) run_item<3, true, STAGE_T10, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                else run_item<3, false, STAGE_T10, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                continue;
            }
        }
        if constexpr ((SET & kBatchSetHalves) != 0) {
            if (d.flags & kFlagHalves) {
                if (neg) run_item<2, true, STAGE_HALVES, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                else run_item<2, false, STAGE_HALVES, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                continue;
            }
        }
        if constexpr (L >= 2 && (SET & kBatchSetCodes)) {
            if (d.flags & kFlagCodes) {
                if (neg) run_item<L, true, STAGE_CODES, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                else run_item<L, false, STAGE_CODES, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                continue;
            }
        }
        if constexpr ((SET & kBatchSetValues) != 0) {
            if ((d.flags & kFlagDirect) == 0) {
                if (neg) run_item<L, true, STAGE_LDS, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                else run_item<L, false, STAGE_LDS, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
            } else {
                if (neg) run_item<L, true, STAGE_DIRECT, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
                else run_item<L, false, STAGE_DIRECT, COUNT>(d, heads, it.i0, it.np, it.t0, it.t1, tile, cnt, steps);
            }
        }
    }
    if (COUNT && (threadIdx.x & (kWave - 1)) == 0 && steps)
        atomicAdd(step_counter, (unsigned long long)steps);
}

// ---------------------------------------------------------------------------
// Kernel selection.
// ---------------------------------------------------------------------------
template <int L, bool NEG, int STAGE, bool COUNT>
const void *eval_ptr()
{
    return reinterpret_cast<const void *>(&k_eval<L, NEG, STAGE, COUNT>);
}

template <bool NEG, int STAGE, bool COUNT>
const void *eval_pick_L(int L)
{
    switch (L) {
    case 1: return eval_ptr<1, NEG, STAGE, COUNT>();
    case 2: return eval_ptr<2, NEG, STAGE, COUNT>();
    case 4: return eval_ptr<4, NEG, STAGE, COUNT>();
    default: return nullptr;
    }
}

template <bool NEG, bool COUNT>
const void *eval_pick_codes(int L)
{
    switch (L) {
    case 2: return eval_ptr<2, NEG, STAGE_CODES, COUNT>();
    case 4: return eval_ptr<4, NEG, STAGE_CODES, COUNT>();
    default: return nullptr;  // codes are staged for 2 or 4 sub-tiles only
    }
}

template <bool COUNT>
const void *eval_pick(int L, bool neg, int staging)
{
    if (staging == STAGE_BYTES) {  // one or two 256-row groups per chunk
        if (L == 4) return neg ? eval_ptr<4, true, STAGE_BYTES, COUNT>() : eval_ptr<4, false, STAGE_BYTES, COUNT>();
        if (L == 8) return neg ? eval_ptr<8, true, STAGE_BYTES, COUNT>() : eval_ptr<8, false, STAGE_BYTES, COUNT>();
        if (L == 16) return neg ? eval_ptr<16, true, STAGE_BYTES, COUNT>() : eval_ptr<16, false, STAGE_BYTES, COUNT>();
        return nullptr;
    }
    if (staging == STAGE_T10) {  // one or two lane words of three rows per chunk
        if (L == 3) return neg ? eval_ptr<3, true, STAGE_T10, COUNT>() : eval_ptr<3, false, STAGE_T10, COUNT>();
        if (L == 6) return neg ? eval_ptr<6, true, STAGE_T10, COUNT>() : eval_ptr<6, false, STAGE_T10, COUNT>();
        return nullptr;
    }
    if (staging == STAGE_HALVES) {  // one or two lane words of two rows per chunk
        if (L == 2) return neg ? eval_ptr<2, true, STAGE_HALVES, COUNT>() : eval_ptr<2, false, STAGE_HALVES, COUNT>();
        if (L == 4) return neg ? eval_ptr<4, true, STAGE_HALVES, COUNT>() : eval_ptr<4, false, STAGE_HALVES, COUNT>();
        return nullptr;
    }
    if (staging == STAGE_CODES) return neg ? eval_pick_codes<true, COUNT>(L) : eval_pick_codes<false, COUNT>(L);
    if (staging == STAGE_LDS)
        return neg ? eval_pick_L<true, STAGE_LDS, COUNT>(L) : eval_pick_L<false, STAGE_LDS, COUNT>(L);
    return neg ? eval_pick_L<true, STAGE_DIRECT, COUNT>(L) : eval_pick_L<false, STAGE_DIRECT, COUNT>(L);
}

const void *eval_kernel(int L, uint32_t flags, int staging, bool count)
{
    const bool neg = (flags & kFlagNeg) != 0;
    return count ? eval_pick<true>(L, neg, staging) : eval_pick<false>(L, neg, staging);
}

const void *batch_kernel(int L, int set, bool count)
{
    // Instances for one kind of SWAR codes (whatever L the other stagings
    // would take), else the general one of each L.
    if (set == kBatchSetBytes)
        return count ? (const void *)&k_eval_batch<2, kBatchSetBytes, true>
                     : (const void *)&k_eval_batch<2, kBatchSetBytes, false>;
    if (set == kBatchSetHalves)
        return count ? (const void *)&k_eval_batch<2, kBatchSetHalves, true>
                     : (const void *)&k_eval_batch<2, kBatchSetHalves, false>;
    if (set == kBatchSetT10)
        return count ? (const void *)&k_eval_batch<2, kBatchSetT10, true>
                     : (const void *)&k_eval_batch<2, kBatchSetT10, false>;
    switch (L) {
    case 1: return count ? (const void *)&k_eval_batch<1, kBatchSetAll, true> : (const void *)&k_eval_batch<1, kBatchSetAll, false>;
    case 2: return count ? (const void *)&k_eval_batch<2, kBatchSetAll, true> : (const void *)&k_eval_batch<2, kBatchSetAll, false>;
    case 4: return count ? (const void *)&k_eval_batch<4, kBatchSetAll, true> : (const void *)&k_eval_batch<4, kBatchSetAll, false>;
    default: return nullptr;
    }
}

hipError_t set_lds(const void *k, size_t lds)
{
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace

size_t tile_lds_bytes(int32_t L, int32_t cols, int32_t staging) { return tile_bytes_of(L, cols, staging); }

size_t count_lds_bytes(int32_t P) { return count_bytes_of(P); }

size_t item_lds_bytes(int32_t L, int32_t cols, int32_t staging, int32_t P, bool cnt16)
{
    return tile_bytes_of(L, cols, staging) + count_bytes_of(P, cnt16);
}

int eval_occupancy(const LaunchCfg &cfg, int32_t cols, uint32_t flags)
{
    const void *k = eval_kernel(cfg.L, flags, cfg.staging, false);
    if (!k) return 0;
    const size_t lds = item_lds_bytes(cfg.L, cols, cfg.staging, cfg.P, cfg.cnt16);
    int blocks = 0;
    if (set_lds(k, lds) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, cfg.W * kWave, lds) != hipSuccess)
        return 0;
    return blocks;
}

int batch_occupancy(int32_t L, int32_t set, int32_t W, size_t lds)
{
    const void *k = batch_kernel(L, set, false);
    if (!k) return 0;
    int blocks = 0;
    if (set_lds(k, lds) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, W * kWave, lds) != hipSuccess) return 0;
    return blocks;
}

hipError_t launch_eval(const ReqDesc &d, IndHead *heads, const LaunchCfg &cfg,
                       unsigned long long *step_counter, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1)
{
    if (d.n <= 0) return hipSuccess;
    if (cfg.staging == STAGE_PAIRS) {
        hipError_t e = launch_prep_pairs(d, heads, s);
        if (e != hipSuccess) return e;
    } else {
        const int threads = 256;
        const int per_block = threads / kWave;  // one wave per individual
        clear_last_error();
        hipLaunchKernelGGL(k_prep, dim3((d.n + per_block - 1) / per_block), dim3(threads), 0, s, d, heads);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (cfg.staging == STAGE_PAIRS) {
        // (no tile and no LDS: a flat grid of chunk x group blocks)
        const void *kp = pairs_kernel(d.flags, step_counter != nullptr, cfg.P, cfg.W);
        const size_t lds = 0;
        hipError_t e = set_lds(kp, lds);
        if (e != hipSuccess) return e;
        // (at most 64 individuals per wave)
        if (cfg.P > 64 * cfg.W) return hipErrorInvalidValue;
        ReqDesc dd = d;
        const IndHead *hh = heads;
        int32_t P = cfg.P, nt = (int32_t)((d.rows + 63) / 64);
        unsigned long long *sc = step_counter;
        void *params[] = {&dd, &hh, &P, &nt, &sc};
        if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
        const dim3 grid = pairs_grid(d.rows, d.n, cfg.P);
        if (grid.x > 0x7fffffffu || grid.y > 65535u) return hipErrorInvalidValue;
        e = hipLaunchKernel(kp, grid, dim3(cfg.W * kWave), params, lds, s);
        if (e != hipSuccess) return e;
        if (ev1) e = hipEventRecord(ev1, s);
        return e;
    }
    // Four words per row group make counts only (no mask outputs).
    if (cfg.L == 16 && (d.mmask || d.nmask)) return hipErrorInvalidValue;
    const void *k = eval_kernel(cfg.L, d.flags, cfg.staging, step_counter != nullptr);
    if (!k) return hipErrorInvalidValue;
    const int32_t n_tiles = (int32_t)((d.rows + 63) / 64);
    const int32_t groups = (d.n + cfg.P - 1) / cfg.P;
    const size_t lds = item_lds_bytes(cfg.L, d.cols, cfg.staging, cfg.P, cfg.cnt16);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    ReqDesc dd = d;
    const IndHead *hh = heads;
    int32_t P = cfg.P, nt = n_tiles;
    unsigned long long *sc = step_counter;
    void *params[] = {&dd, &hh, &P, &nt, &sc};
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
    e = hipLaunchKernel(k, dim3(cfg.blocks, groups), dim3(cfg.W * kWave), params, lds, s);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, s);
    return e;
}

}  // namespace ebic

// ---------------------------------------------------------------------------
// The fixed header buffer of ebic_eval_population_noalloc: room for the
// 64-byte headers of kNoAllocMaxInd individuals, one copy per device (each
// device that loads this code object holds its own, until the process
// ends). Host code never passes the array's name to a kernel: it takes the
// device address from hipGetSymbolAddress once per device and uses that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) ebic::IndHead scratch[ebic::kNoAllocMaxInd];

namespace ebic {

namespace {
std::mutex g_noalloc_mu;
std::map<int, void *> g_noalloc_ptr;  // device -> address of `scratch` there
}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr.count(device)) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_noalloc_ptr[device] = ptr;
    return hipSuccess;
}

IndHead *noalloc_scratch(int device)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc_ptr.find(device);
    return it == g_noalloc_ptr.end() ? nullptr : static_cast<IndHead *>(it->second);
}

hipError_t launch_batch(BatchHeader *hdr, const ReqDesc *descs, const int64_t *first,
                        const Item *items, IndHead *heads, int32_t L, int32_t set, int32_t W, int32_t P,
                        size_t tile_bytes, int32_t grid, int32_t prep_blocks,
                        unsigned long long *step_counter, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1)
{
    clear_last_error();
    hipLaunchKernelGGL(k_prep_batch, dim3(prep_blocks), dim3(256), 0, s, hdr, descs, first, heads);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (grid <= 0) return hipSuccess;  // (no request on the tiled kernel)
    const void *k = batch_kernel(L, set, step_counter != nullptr);
    if (!k) return hipErrorInvalidValue;
    const size_t lds = tile_bytes + count_bytes_of(P);
    if ((e = set_lds(k, lds)) != hipSuccess) return e;
    BatchHeader *h = hdr;
    const ReqDesc *dd = descs;
    const Item *it = items;
    const IndHead *hh = heads;
    int32_t tb = (int32_t)tile_bytes;
    int32_t PP = P;
    unsigned long long *sc = step_counter;
    void *params[] = {&h, &dd, &it, &hh, &tb, &PP, &sc};
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
    e = hipLaunchKernel(k, dim3(grid), dim3(W * kWave), params, lds, s);
    if (e != hipSuccess) return e;
    if (ev1) e = hipEventRecord(ev1, s);
    return e;
}

}  // namespace ebic

// ebic_pairs.hip -- the predicate over pairwise order bitmaps.
//
// The trend relation of an individual (c_0, ..., c_{k-1}) on a row holds
// when every consecutive pair does: x[r, c_j] >= x[r, c_{j-1}] for the
// positive chain, x[r, c_{j-1}] >= x[r, c_j] for the reversed one (Methods,
// "Handling missing values": the rows are counted by this relation). Both
// chains are conjunctions over the individual's consecutive column pairs,
// and there are only cols^2 ordered pairs. So the library can compare every
// ordered pair of columns once per row, on first use, and keep the answers
// as bitmaps:
//
//   G[a * cols + b] bit r  =  x[r, b] >= x[r, a]      (IEEE single: a NaN
//                                                       on either side is 0)
//
// The diagonal pair (a, a) is then "x[r, a] is present". An individual's
// positive chain on 32 rows is one AND per pair of one 32-bit word per
// lane, its reversed chain the same over the reversed pairs, and a row
// matched by both directions (constant along the individual) counts once,
// as positive. The results are those of the comparisons themselves, bit for
// bit: the bitmaps hold the compares' outcomes, ties and signed zeros
// included.
//
// Layout: chunk by chunk (2,048 rows: one 32-bit word per lane of a wave),
// and within a chunk pair by pair, pair (a, b) of chunk q at word
// ((q * cols + a) * cols + b) * 64; bit i of a lane's word is row
// 2048 q + 32 lane + i. Rows past the matrix are 0. A chunk's pairs span
// cols^2 x 256 bytes, so a wave addresses them with 32-bit offsets from the
// chunk's base. Include mode reads a second set built from the
// fill-substituted values (the same set when no cell is missing).
//
// Behind the bitmaps, 512 bytes per chunk list its ties: word 0 counts the
// entries, word 1 is non-zero if a NaN occurs in the chunk, and words
// 64 .. 127 hold the byte offsets of both orders of each pair of different
// columns with two equal values on some row (up to 32 pairs; a count past
// 64 means more). Where a chunk has no NaN and a pair (a, b), a != b, is not
// listed, every row has x_a, x_b present and distinct, so the reversed
// pair's word is the complement of the pair's on the matrix's rows: the
// reversed chain then needs no loads of its own.
//
// Evaluation: a block per (group of individuals, chunk), its waves taking
// the group's individuals in turn. A prep kernel writes each individual's
// 64-byte pairs header: k, the CSR start, the byte offsets of the pairs of
// its first eight columns (consecutive repeats left out: a pair (c, c) is
// implied by the pairs next to it, and the first pair is of two different
// columns), and the window's columns. Per individual and chunk the wave
// loads the seven pairs (two individuals' at a time), ANDs them, takes the
// reversed chain as their complement where the chunk allows it (else loads
// the reversed pairs), and follows the columns past the window eight at a
// time while any row is left. Where a wave takes many individuals per item
// (the batched kernel, and plain launches of eight or more per wave), the
// next two individuals' headers are loaded while the current pairs are in
// flight. No tile is staged: the words come through L2
// and the Infinity Cache, where the pairs shared by the individuals of a
// chunk are reused, and the blocks of a chunk are placed on one XCD and run
// together. The counts of the wave's 2,048 rows are summed across lanes by
// DPP (row shifts, then row broadcasts) into a lane of the wave's own, and
// added to the outputs once per item.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ebic_internal.h"
#include "ebic_prep.h"

namespace ebic {
namespace {

constexpr int kChunkRows = 2048;  // rows per wave step: 64 lanes x 32 rows
constexpr int kChunkWords = 64;
constexpr int kTieWords = 128;    // per chunk: count, NaN flag, ..., 64 listed offsets
constexpr int kTieList = 64;      // (the list's first word)
constexpr uint32_t kNoPair = 0xffffffffu;  // never a pair's offset (those are multiples of 256)
constexpr int kPipeMin = 8;       // individuals per wave and item from which the headers are loaded ahead

__global__ void __launch_bounds__(256) k_prep_pairs(ReqDesc d, IndHead *__restrict__ heads)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int32_t i = blockIdx.x * (blockDim.x / kWave) + wave;
    if (i < d.n) prep_pairs_wave(d, i, heads, threadIdx.x & (kWave - 1));
}

// One wave per block: columns a0 = A t .. A t + A - 1 of one chunk against
// every b >= a0, the words of pairs (a, b) and (b, a) on the chunk's rows;
// lane l covers rows chunk*2048 + 32 l ... + 31 (one 128-byte run of each
// column), and each column b is loaded once for the block's A columns. Ties
// and NaN go to the chunk's list (T, zeroed beforehand). The grid is
// (8 x ceil(cols / A), chunks / 8): block (x, y) takes chunk 8 y + x mod 8
// and t = x / 8, so a chunk's blocks all run on one XCD, one after another,
// and its columns stay in that XCD's L2 while they do.
template <int A>
__global__ void __launch_bounds__(64) k_pair_bits(const float *__restrict__ X, int64_t rows, int64_t ld,
                                                  int32_t cols, int32_t subst, float fill,
                                                  uint32_t *__restrict__ G, uint32_t *__restrict__ T)
{
    const int64_t n_chunks = (rows + kChunkRows - 1) / kChunkRows;
    const int64_t chunk = 8 * (int64_t)blockIdx.y + (blockIdx.x & 7);
    const int32_t a0 = A * (int32_t)(blockIdx.x >> 3);
    if (chunk >= n_chunks || a0 >= cols) return;
    const int lane = (int)threadIdx.x;
    const int64_t r0 = chunk * kChunkRows + 32 * lane;
    // valid rows of this lane's 32 as a bit mask
    const int64_t nvalid = rows - r0;
    const uint32_t vmask = nvalid >= 32 ? 0xffffffffu : nvalid <= 0 ? 0u : ((1u << nvalid) - 1u);
    auto load32 = [&](int32_t c, float (&v)[32]) {
        if (r0 < ld) {
            const float4 *p = reinterpret_cast<const float4 *>(X + (int64_t)c * ld + r0);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 f = p[q];
                v[4 * q] = f.x;
                v[4 * q + 1] = f.y;
                v[4 * q + 2] = f.z;
                v[4 * q + 3] = f.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 32; ++i) v[i] = __builtin_nanf("");
        }
        if (subst) {
#pragma unroll
            for (int i = 0; i < 32; ++i) v[i] = v[i] != v[i] ? fill : v[i];
        }
    };
    uint32_t *tl = T + chunk * kTieWords;
    const uint32_t cb = (uint32_t)cols * 256u;
    // the words of pairs (a, b) and (b, a), b >= a
    auto emit = [&](int32_t a, const float (&xa)[32], int32_t b, const float (&xb)[32]) {
        uint32_t ge = 0, le = 0;  // x_b >= x_a, x_a >= x_b
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            ge |= (xb[i] >= xa[i] ? 1u : 0u) << i;
            le |= (xa[i] >= xb[i] ? 1u : 0u) << i;
        }
        G[((chunk * cols + a) * cols + b) * kChunkWords + lane] = ge & vmask;
        if (b != a) G[((chunk * cols + b) * cols + a) * kChunkWords + lane] = le & vmask;
        const uint32_t odd = (b == a ? ~ge : (ge & le)) & vmask;  // NaN rows; tied rows
        if (__ballot(odd != 0) != 0 && lane == 0) {
            if (b == a) {
                atomicOr(tl + 1, 1u);
            } else {
                const uint32_t slot = atomicAdd(tl, 2u);
                if (slot + 2 <= (uint32_t)kTieList) {
                    tl[kTieList + slot] = (uint32_t)a * cb + ((uint32_t)b << 8);
                    tl[kTieList + slot + 1] = (uint32_t)b * cb + ((uint32_t)a << 8);
                }
            }
        }
    };
    float xa[A][32];
#pragma unroll
    for (int j = 0; j < A; ++j) load32(min(a0 + j, cols - 1), xa[j]);
    for (int32_t b = a0; b < cols; ++b) {
        float xb[32];
        load32(b, xb);
#pragma unroll
        for (int j = 0; j < A; ++j)
            if (b >= a0 + j) emit(a0 + j, xa[j], b, xb);
    }
}

// Sum over the wave's 64 lanes, returned to every lane: an inclusive scan
// within each row of 16 lanes (row shifts by 1, 2, 4, 8), then row 0's
// total added into row 1 and row 2's into row 3 (row broadcast of lane 15),
// then lane 31's into rows 2 and 3 (row broadcast of lane 31): lane 63 holds
// the sum.
__device__ __forceinline__ uint32_t wave_total(uint32_t v)
{
    int s = (int)v;
    s += __builtin_amdgcn_update_dpp(0, s, 0x111, 0xf, 0xf, true);   // row_shr:1
    s += __builtin_amdgcn_update_dpp(0, s, 0x112, 0xf, 0xf, true);   // row_shr:2
    s += __builtin_amdgcn_update_dpp(0, s, 0x114, 0xf, 0xf, true);   // row_shr:4
    s += __builtin_amdgcn_update_dpp(0, s, 0x118, 0xf, 0xf, true);   // row_shr:8
    s += __builtin_amdgcn_update_dpp(0, s, 0x142, 0xa, 0xf, false);  // row_bcast:15
    s += __builtin_amdgcn_update_dpp(0, s, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane(s, 63);
}

// What the item loop takes from a pairs header up front (the CSR start and
// the window's columns are read where they are needed: the reversed pairs'
// loads and the columns past the window).
struct PairScal {
    int32_t k;
    uint32_t f[7];
};

__device__ __forceinline__ PairScal pair_scal(const PairHead *h)
{
    const int4 *p = reinterpret_cast<const int4 *>(h);
    const int4 x0 = p[0], x1 = p[1];
    const uint32_t x2 = h->fwd[6];
    PairScal s;
    s.k = __builtin_amdgcn_readfirstlane(x0.x);
    s.f[0] = (uint32_t)__builtin_amdgcn_readfirstlane(x0.z);
    s.f[1] = (uint32_t)__builtin_amdgcn_readfirstlane(x0.w);
    s.f[2] = (uint32_t)__builtin_amdgcn_readfirstlane(x1.x);
    s.f[3] = (uint32_t)__builtin_amdgcn_readfirstlane(x1.y);
    s.f[4] = (uint32_t)__builtin_amdgcn_readfirstlane(x1.z);
    s.f[5] = (uint32_t)__builtin_amdgcn_readfirstlane(x1.w);
    s.f[6] = (uint32_t)__builtin_amdgcn_readfirstlane((int)x2);
    return s;
}

// One work item: individuals [i0, i0 + np) of a request on one 2,048-row
// chunk, by the W waves of a block (the wave's individuals in turn, at most
// 64 per wave); each lane of a wave keeps the counts of one of the wave's
// individuals, added to the outputs at the end.
template <bool NEG, bool COUNT, bool PIPE>
__device__ __forceinline__ void pairs_item(const ReqDesc &d, const IndHead *__restrict__ heads, int32_t i0,
                                           int32_t np, int32_t chunk, int lane, int wave, int W, uint64_t &steps)
{
    const int32_t C = d.cols;
    const uint32_t cb = (uint32_t)C * 256u;  // pairs (a, 0 .. C-1) of a chunk
    const int voff = lane * 4;
    const PairHead *hb = reinterpret_cast<const PairHead *>(heads + d.head_base + i0);
    // mask words (as 32-bit halves, little-endian: the uint64 layout)
    const int64_t words32 = 2 * ((d.rows + 63) / 64);
    const bool masks = d.mmask || d.nmask;
    uint32_t acc_m = 0, acc_g = 0;  // lane t: the wave's t-th individual

    {
        const uint32_t *gchunk = reinterpret_cast<const uint32_t *>(d.B) + (int64_t)chunk * C * C * kChunkWords;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(gchunk), (short)0, C * C * 256, 0x00020000);
        // pair (a, c) of the chunk, this lane's word: offset a * C * 256 + c * 256
        auto ld = [&](uint32_t off) { return __builtin_amdgcn_raw_buffer_load_b32(rs, voff, (int)off, 0); };
        // The chunk's ties: lane l holds listed offset l (kNoPair past the
        // count); `dirty` when the list overflowed or a NaN occurs.
        const uint32_t *tl = reinterpret_cast<const uint32_t *>(d.T) + (int64_t)chunk * kTieWords;
        const uint32_t n_tied = __builtin_amdgcn_readfirstlane(tl[0]);
        const uint32_t nan_flag = __builtin_amdgcn_readfirstlane(tl[1]);  // (read either way: no dependent load)
        const bool dirty = (n_tied > (uint32_t)kTieList) | (nan_flag != 0);
        const uint32_t tied = (uint32_t)lane < n_tied ? tl[kTieList + lane] : kNoPair;
        const bool clean = n_tied == 0 && !dirty;
        const int64_t nvalid = d.rows - ((int64_t)chunk * kChunkRows + 32 * lane);
        const uint32_t vmask = nvalid >= 32 ? 0xffffffffu : nvalid <= 0 ? 0u : ((1u << nvalid) - 1u);
        // may the reversed chain over these pair offsets be the complement?
        auto untied = [&](const uint32_t *off, int n) {
            if (clean) return true;
            if (dirty) return false;
            bool hit = false;
            for (int t = 0; t < n; ++t) hit |= tied == off[t];
            return __ballot(hit) == 0;
        };
        const int64_t word = (int64_t)chunk * kChunkWords + lane;
        const bool store = word < words32;

        // The reversed chain of the window from its columns (loads of the
        // reversed pairs; (c, c): "present", implied by the pairs next to it).
        auto slow_window = [&](const PairHead *h) {
            const uint32_t *hw = h->win;
            uint32_t wp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) wp[u] = (uint32_t)__builtin_amdgcn_readfirstlane((int)hw[u]);
            uint32_t q[7];
#pragma unroll
            for (int u = 0; u < 7; ++u) {
                const uint32_t a = (wp[u >> 1] >> ((u & 1) * 16)) & 0xffffu;
                const uint32_t c = (wp[(u + 1) >> 1] >> (((u + 1) & 1) * 16)) & 0xffffu;
                q[u] = ld(c * cb + (a << 8));
            }
            return q[0] & q[1] & q[2] & q[3] & q[4] & q[5] & q[6];
        };
        // The columns past the window, eight at a time (the last one
        // repeated past the end), while a row is left.
        auto tail = [&](uint32_t &Pw, uint32_t &Nw, int32_t k, const PairHead *h) {
            const int32_t *cc = d.colidx + __builtin_amdgcn_readfirstlane(h->begin);
            uint32_t prev = (uint32_t)__builtin_amdgcn_readfirstlane((int)h->win[3]) >> 16;  // the window's last column
            for (int32_t u = 8; u < k; u += 8) {
                uint32_t cn[8], fo[8], pp[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) cn[e] = (uint32_t)__builtin_amdgcn_readfirstlane(cc[min(u + e, k - 1)]);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    fo[e] = (e == 0 ? prev : cn[e - 1]) * cb + (cn[e] << 8);
                    pp[e] = ld(fo[e]);
                }
                Pw &= pp[0] & pp[1] & pp[2] & pp[3] & pp[4] & pp[5] & pp[6] & pp[7];
                if (NEG) {
                    if (untied(fo, 8)) {
                        // (c, c) pairs: "present", all the chunk's rows
                        uint32_t nq = 0;
#pragma unroll
                        for (int e = 0; e < 8; ++e) nq |= (e == 0 ? prev : cn[e - 1]) == cn[e] ? 0u : pp[e];
                        Nw &= ~nq;
                    } else {
                        uint32_t qq[8];
#pragma unroll
                        for (int e = 0; e < 8; ++e) qq[e] = ld(cn[e] * cb + ((e == 0 ? prev : cn[e - 1]) << 8));
                        Nw &= qq[0] & qq[1] & qq[2] & qq[3] & qq[4] & qq[5] & qq[6] & qq[7];
                    }
                }
                prev = cn[7];
                if (COUNT) steps += (uint64_t)min(8, k - u);
                if (__ballot((Pw | Nw) != 0) == 0) break;
            }
        };
        // Masks and counts of the wave's t-th individual (ii).
        auto finish = [&](uint32_t Pw, uint32_t Nw, int32_t ii, int32_t t) {
            const uint32_t mw = Pw | Nw, gw = NEG ? (Nw & ~Pw) : 0u;
            if (masks && store) {
                if (d.mmask) reinterpret_cast<uint32_t *>(d.mmask)[(int64_t)(i0 + ii) * words32 + word] = mw;
                if (d.nmask) reinterpret_cast<uint32_t *>(d.nmask)[(int64_t)(i0 + ii) * words32 + word] = gw;
            }
            if (__ballot(mw != 0) == 0) return;
            const uint32_t both =
                wave_total((uint32_t)__builtin_popcount(mw) | ((uint32_t)__builtin_popcount(gw) << 16));
            if (lane == t) {
                acc_m += both & 0xffffu;
                if (NEG) acc_g += both >> 16;
            }
        };

        // Two individuals at a time (ii and ii + W, the wave's t-th and
        // (t + 1)-th): both windows' loads in flight together, and the
        // next two individuals' headers loaded while they are. The window
        // needs no branch: an individual of one column has the diagonal
        // pair in every slot (its reversed chain, whatever it gives, adds
        // nothing: its rows are all positive), and an invalid one (k = 0)
        // is zeroed after the loads.
        int32_t ii = wave;
        if (ii < np) {
            int32_t t = 0;
            PairScal A = pair_scal(hb + ii), B = pair_scal(hb + min(ii + W, np - 1));
            for (;;) {
                const bool two = ii + W < np;
                uint32_t pa[7], pb[7];
#pragma unroll
                for (int u = 0; u < 7; ++u) {
                    pa[u] = ld(A.f[u]);
                    pb[u] = ld(B.f[u]);
                }
                const int32_t jn = ii + 2 * W;
                const bool more = jn < np;
                PairScal An, Bn;
                if (PIPE && more) {
                    An = pair_scal(hb + jn);
                    Bn = pair_scal(hb + min(jn + W, np - 1));
                }
                uint32_t Pa = pa[0] & pa[1] & pa[2] & pa[3] & pa[4] & pa[5] & pa[6];
                uint32_t Pb = pb[0] & pb[1] & pb[2] & pb[3] & pb[4] & pb[5] & pb[6];
                uint32_t Na = 0, Nb = 0;
                if (NEG) {
                    Na = untied(A.f, 7) ? ~(pa[0] | pa[1] | pa[2] | pa[3] | pa[4] | pa[5] | pa[6]) & vmask
                                        : slow_window(hb + ii);
                    Nb = untied(B.f, 7) ? ~(pb[0] | pb[1] | pb[2] | pb[3] | pb[4] | pb[5] | pb[6]) & vmask
                                        : slow_window(hb + min(ii + W, np - 1));
                }
                if (A.k == 0) Pa = Na = 0u;
                if (B.k == 0) Pb = Nb = 0u;
                if (COUNT) steps += (A.k > 1 ? 7 : A.k) + (two ? (B.k > 1 ? 7 : B.k) : 0);
                if (A.k > 8 && __ballot((Pa | Na) != 0) != 0) tail(Pa, Na, A.k, hb + ii);
                finish(Pa, Na, ii, t);
                if (two) {
                    if (B.k > 8 && __ballot((Pb | Nb) != 0) != 0)
                        tail(Pb, Nb, B.k, hb + ii + W);
                    finish(Pb, Nb, ii + W, t + 1);
                }
                if (!more) break;
                if (PIPE) {
                    A = An;
                    B = Bn;
                } else {
                    A = pair_scal(hb + jn);
                    B = pair_scal(hb + min(jn + W, np - 1));
                }
                ii = jn;
                t += 2;
            }
        }
    }
    // the wave's individuals wave + t W, t = lane
    const int32_t ii = wave + lane * W;
    if (ii < np) {
        if (acc_m) atomicAdd(d.matched + i0 + ii, (int32_t)acc_m);
        if (NEG && acc_g && d.negative) atomicAdd(d.negative + i0 + ii, (int32_t)acc_g);
    }
}

// The plain launch: a 2-D grid of (8 x groups, chunks / 8) blocks. Block
// (x, y) works on chunk 8 y + x mod 8 and group x / 8: blocks are dispatched
// x first, and with gridDim.x a multiple of 8 the linear block index is
// x mod 8 modulo 8, so on MI355X's round-robin placement of blocks over the
// eight XCDs the blocks of a chunk all run on one XCD and share its L2, and
// the blocks of eight consecutive chunks (all their groups) are dispatched
// together.
template <bool NEG, bool COUNT, bool PIPE>
__global__ void __launch_bounds__(1024) k_eval_pairs(ReqDesc d, const IndHead *__restrict__ heads, int32_t P,
                                                     int32_t n_tiles, unsigned long long *step_counter)
{
    const int32_t n_chunks = (n_tiles + 31) / 32;
    const int32_t chunk = (int32_t)(8 * blockIdx.y + (blockIdx.x & 7));
    const int32_t grp = (int32_t)(blockIdx.x >> 3);
    if (chunk >= n_chunks) return;
    const int32_t i0 = grp * P;
    const int32_t np = min(P, d.n - i0);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    uint64_t steps = 0;
    pairs_item<NEG, COUNT, PIPE>(d, heads, i0, np, chunk, lane, wave, blockDim.x / kWave, steps);
    if (COUNT && lane == 0 && steps) atomicAdd(step_counter, (unsigned long long)steps);
}

// The batched launch: a fixed grid (a multiple of 8 blocks) over eight item
// lists, one per XCD slice: block b walks list b mod 8 with a stride of
// grid / 8 (items b / 8, b / 8 + grid / 8, ...), so the blocks of a slice
// take its items in order, all of them near the same chunk at a time, with
// no counter to contend for. A list walks its slice's chunks in order,
// segment by segment (the requests that read one set of bitmaps), every
// group of every request of the segment on a chunk before the next chunk:
// item k of slice x in segment g is chunk 8 (l / groups) + x and group
// l mod groups (l = k minus the segment's first item in the list), the
// group found among the segment's requests by their first groups.
template <bool COUNT>
__global__ void __launch_bounds__(1024) k_eval_pairs_batch(const PairQueues *__restrict__ pq,
                                                           const ReqDesc *__restrict__ descs,
                                                           const PairSeg *__restrict__ segs,
                                                           const int32_t *__restrict__ seg_req,
                                                           const int32_t *__restrict__ seg_gstart,
                                                           const IndHead *__restrict__ heads,
                                                           unsigned long long *step_counter)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int W = blockDim.x / kWave;
    const int32_t n_seg = pq->n_seg;
    const int32_t P = min(pq->P, 64 * W);  // (the planner keeps it there)
    const int slice = (int)(blockIdx.x % 8);
    const int32_t stride = (int32_t)(gridDim.x / 8);
    const int32_t total = pq->total[slice];
    uint64_t steps = 0;
    int32_t g = 0;  // (items come in order: the segment only moves forward)
    for (int32_t k = (int32_t)(blockIdx.x / 8); k < total; k += stride) {
        while (g + 1 < n_seg && segs[g + 1].base[slice] <= k) ++g;
        const int32_t local = k - segs[g].base[slice];
        const int32_t groups = segs[g].groups;
        const int32_t chunk = 8 * (local / groups) + slice;
        const int32_t pos = local % groups;
        int32_t lo = segs[g].e0, hi = segs[g].e0 + segs[g].n_req - 1;  // the last entry starting at or before pos
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (seg_gstart[mid] <= pos) lo = mid;
            else hi = mid - 1;
        }
        const ReqDesc &d = descs[seg_req[lo]];
        const int32_t i0 = (pos - seg_gstart[lo]) * P;
        const int32_t np = min(P, d.n - i0);
        if (d.flags & kFlagNeg) pairs_item<true, COUNT, true>(d, heads, i0, np, chunk, lane, wave, W, steps);
        else pairs_item<false, COUNT, true>(d, heads, i0, np, chunk, lane, wave, W, steps);
    }
    if (COUNT && lane == 0 && steps) atomicAdd(step_counter, (unsigned long long)steps);
}

}  // namespace

int64_t pair_words(int64_t rows) { return (rows + kChunkRows - 1) / kChunkRows * kChunkWords; }

int64_t pair_tie_bytes(int64_t rows)
{
    return (rows + kChunkRows - 1) / kChunkRows * kTieWords * (int64_t)sizeof(uint32_t);
}

hipError_t launch_pair_bits(const float *X, int64_t rows, int64_t ld, int32_t cols, bool subst, float fill,
                            uint32_t *G, int64_t w32, uint32_t *T, hipStream_t s)
{
    if (cols < 1 || cols > kMaxPairCols || w32 != pair_words(rows) || ld % 64 != 0) return hipErrorInvalidValue;
    const int64_t chunks = w32 / kChunkWords;
    const int64_t per_slice = (chunks + 7) / 8;
    if (per_slice > 65535) return hipErrorInvalidValue;
    // Four columns per block past 128 columns (the loads of each b shared
    // four ways), two below, where fewer blocks per chunk would be left.
    const bool four = cols > 128;
    const int A = four ? 4 : 2;
    const dim3 grid((unsigned)(8 * ((cols + A - 1) / A)), (unsigned)per_slice);
    const int sub = subst ? 1 : 0;
    clear_last_error();
    if (four) hipLaunchKernelGGL(k_pair_bits<4>, grid, dim3(64), 0, s, X, rows, ld, cols, sub, fill, G, T);
    else hipLaunchKernelGGL(k_pair_bits<2>, grid, dim3(64), 0, s, X, rows, ld, cols, sub, fill, G, T);
    return hipGetLastError();
}

hipError_t launch_prep_pairs(const ReqDesc &d, IndHead *heads, hipStream_t s)
{
    const int threads = 256;
    const int per_block = threads / kWave;  // one wave per individual
    clear_last_error();
    hipLaunchKernelGGL(k_prep_pairs, dim3((d.n + per_block - 1) / per_block), dim3(threads), 0, s, d, heads);
    return hipGetLastError();
}

static const void *pairs_batch_kernel(bool count)
{
    return count ? (const void *)&k_eval_pairs_batch<true> : (const void *)&k_eval_pairs_batch<false>;
}

int pairs_batch_occupancy(int32_t W)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, pairs_batch_kernel(false), W * kWave, 0) != hipSuccess)
        return 0;
    return blocks;
}

hipError_t launch_pairs_batch(const PairQueues *pq, const ReqDesc *descs, const PairSeg *segs,
                              const int32_t *seg_req, const int32_t *seg_gstart, const IndHead *heads, int32_t W,
                              int32_t grid, unsigned long long *step_counter, hipStream_t s)
{
    if (W < 1 || W > 16 || grid < 8 || grid % 8 != 0) return hipErrorInvalidValue;
    const bool count = step_counter != nullptr;
    clear_last_error();
    if (count)
        hipLaunchKernelGGL(k_eval_pairs_batch<true>, dim3(grid), dim3(W * kWave), 0, s, pq, descs, segs, seg_req,
                           seg_gstart, heads, step_counter);
    else
        hipLaunchKernelGGL(k_eval_pairs_batch<false>, dim3(grid), dim3(W * kWave), 0, s, pq, descs, segs, seg_req,
                           seg_gstart, heads, step_counter);
    return hipGetLastError();
}

const void *pairs_kernel(uint32_t flags, bool count, int32_t P, int32_t W)
{
    const bool neg = (flags & kFlagNeg) != 0;
    // Loading the next headers early pays once a wave takes four or more
    // pairs of individuals per item; with fewer, the extra scalar registers
    // cost more than the hidden latency.
    const bool pipe = (P + W - 1) / W >= kPipeMin;
    if (pipe) {
        if (count) return neg ? (const void *)&k_eval_pairs<true, true, true> : (const void *)&k_eval_pairs<false, true, true>;
        return neg ? (const void *)&k_eval_pairs<true, false, true> : (const void *)&k_eval_pairs<false, false, true>;
    }
    if (count) return neg ? (const void *)&k_eval_pairs<true, true, false> : (const void *)&k_eval_pairs<false, true, false>;
    return neg ? (const void *)&k_eval_pairs<true, false, false> : (const void *)&k_eval_pairs<false, false, false>;
}

// The plain pairs launch's grid: (8 x groups, chunks / 8 rounded up).
dim3 pairs_grid(int64_t rows, int32_t n, int32_t P)
{
    const int64_t groups = (n + P - 1) / P;
    const int64_t per_slice = ((rows + kChunkRows - 1) / kChunkRows + 7) / 8;
    return dim3((unsigned)(8 * groups), (unsigned)per_slice);
}

}  // namespace ebic

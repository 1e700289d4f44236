// ebic_prep.h -- the per-individual scan shared by the prep kernels.
//
// One wave per individual: the lanes read its columns together (one round
// of independent loads for up to 64 columns), check every column against
// the matrix width, find the leading run of repeats of the first column,
// and gather the header's window of eight columns.
//
// A leading run of repeats of the first column is dropped from the header
// (begin moves to the run's last entry, k shrinks by the same amount):
// comparing a cell with itself always holds (x >= x and x <= x for any
// present value; a missing one is excluded by the kept copy of the column
// in exclude mode and takes the fill value in include mode), so
// c, c, ..., c, rest follows exactly the rows of c, rest, on both chains.
// The evaluation then never sees a first pair that compares a cell with
// itself, which is what lets a chunk without two equal values in any row
// skip the tie handling of the first pair (the SWAR sequences' tie-free
// variants classify every row as rising or falling there), and what gives
// every individual of two or more columns a first pair of two different
// columns.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ebic_internal.h"

namespace ebic {

constexpr int32_t kInvalid = -1;  // the counts of an individual with an invalid column

struct PrepScan {
    bool ok;      // a non-empty span of valid columns (wave-uniform)
    int32_t k;    // columns from the header's start (0 when not ok)
    int32_t bb;   // the header's CSR start (the last leading repeat)
    int32_t win;  // lanes 8..15: window column lane - 8 from bb (clamped to the last column)
};

__device__ __forceinline__ PrepScan prep_scan(const ReqDesc &d, int32_t i, int lane)
{
    const int32_t b = d.offsets[i], e = d.offsets[i + 1];
    const bool span = b >= 0 && e > b;
    bool bad = false;
    int32_t first = 0;  // lane l: column l of the individual (first 64)
    int32_t run = 0;    // entries b .. b + run hold the first column
    if (span) {
        const int32_t c0 = d.colidx[b];
        run = e - b - 1;  // unless a different column follows
        bool found = false;
        for (int32_t jb = b; jb < e; jb += kWave) {  // (wave-uniform trip count)
            const int32_t j = jb + lane;
            const bool in = j < e;
            const int32_t c = in ? d.colidx[j] : c0;
            if (jb == b) first = c;
            bad |= in && (c < 0 || c >= d.cols);
            const uint64_t differ = __ballot(in && c != c0);
            if (!found && differ != 0) {
                found = true;
                run = (jb - b) + (int32_t)__builtin_ctzll(differ) - 1;
            }
        }
    }
    PrepScan sc;
    sc.ok = span && __ballot(bad) == 0;
    sc.bb = b + run;
    sc.k = sc.ok ? e - sc.bb : 0;
    const int32_t src = run + min(lane - 8, e - sc.bb - 1);
    int32_t win = __shfl(first, (src >= 0 && src < kWave) ? src : 0);
    if (span && lane >= 8 && lane < 16 && src >= kWave) win = d.colidx[b + src];
    sc.win = win;
    return sc;
}

// The pairs header (the IndHead storage, read differently) of the
// pairwise-order-bitmap kernels.
struct PairHead {
    int32_t k;         // columns from begin (0: invalid)
    int32_t begin;     // CSR start (the last leading repeat of the first column)
    uint32_t fwd[7];   // byte offsets of the window's pairs of different columns (the last one repeated);
                       // for k = 1, fwd[0] is the column's diagonal pair
    uint32_t pad0;
    uint32_t win[4];   // the window's eight columns, two per word (low half first)
    uint32_t pad1[2];
};
static_assert(sizeof(PairHead) == sizeof(IndHead), "the pairs header reuses the header storage");

// One wave per individual: the scan, the outputs' initialisation, and the
// pairs header. Lane u < 7 forms window pair (u, u + 1); the pairs of
// different columns are packed to the front in order (a pair (c, c) is
// implied by the pairs next to it), the last one repeating after them; an
// individual of one column gets its diagonal pair ("present").
__device__ __forceinline__ void prep_pairs_wave(const ReqDesc &d, int32_t i, IndHead *__restrict__ heads, int lane)
{
    const PrepScan sc = prep_scan(d, i, lane);
    if (lane == 0) {
        d.matched[i] = sc.ok ? 0 : kInvalid;
        if (d.negative) d.negative[i] = sc.ok ? 0 : kInvalid;
    }
    uint32_t *hd = reinterpret_cast<uint32_t *>(heads + d.head_base + i);
    const uint32_t cb = (uint32_t)d.cols * 256u;  // a pair (a, b)'s byte offset: a * cb + b * 256
    const uint32_t a = (uint32_t)__shfl(sc.win, 8 + min(lane, 7));
    const uint32_t c = (uint32_t)__shfl(sc.win, 8 + min(lane + 1, 7));
    const int q = (lane - 10) & 3;  // lanes 10..13: columns 2q, 2q + 1
    const uint32_t pk = (uint32_t)__shfl(sc.win, 8 + 2 * q) | ((uint32_t)__shfl(sc.win, 9 + 2 * q) << 16);
    const bool distinct = lane < 7 && a != c;
    const uint64_t dm = __ballot(distinct);
    const uint32_t off = a * cb + (c << 8);
    const int nf = __popcll(dm);
    const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)a, 0);
    const uint32_t last = nf == 0 ? w0 * cb + (w0 << 8)
                                  : (uint32_t)__builtin_amdgcn_readlane((int)off, 63 - __clzll(dm));
    if (!sc.ok) {
        if (lane < 16) hd[lane] = 0u;
        return;
    }
    if (distinct) hd[2 + __popcll(dm & ((1ull << lane) - 1))] = off;
    if (lane >= nf && lane < 7) hd[2 + lane] = last;
    if (lane == 0) hd[0] = (uint32_t)sc.k;
    if (lane == 1) hd[1] = (uint32_t)sc.bb;
    if (lane == 9 || lane == 14 || lane == 15) hd[lane] = 0u;
    if (lane >= 10 && lane < 14) hd[lane] = pk;
}

}  // namespace ebic

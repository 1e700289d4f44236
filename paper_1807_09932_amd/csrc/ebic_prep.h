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

}  // namespace ebic

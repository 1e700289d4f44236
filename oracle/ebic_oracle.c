/*
 * ebic_oracle.c -- CPU oracle of EBIC's row-counting fitness evaluation.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The product path
 * (the HIP library and its Python binding) never links, loads or calls it,
 * and the two share no source file, header, helper or table.
 *
 * What it computes (Methods, "Handling missing values"): EBIC's search is
 * driven by counting rows, and a row supports a candidate bicluster when
 * the values in the candidate's columns stand in a greater-or-equal relation.
 * The candidate (an individual of the evolutionary search, Introduction and
 * Methods "Support for Big Data") is an ordered list of column indices
 * c_0 .. c_{k-1}. For each row r, with v_j = X[r, c_j]:
 *
 *   P = AND_{j=1..k-1} (v_j >= v_{j-1})      positive trend, ties allowed
 *   N = NEG AND AND_{j=1..k-1} (v_j <= v_{j-1})  reversed trend (optional)
 *   matched bit  = P or N
 *   negative bit = N and not P              (a row on both is counted once,
 *                                            as positive)
 *
 * Missing values (Methods, "Handling missing values"): a cell is missing when
 * it is NaN or compares equal to the given sentinel (pass NaN for "no
 * sentinel"). In the exclude mode a row with any missing value among the
 * individual's columns is not counted. In the include (legacy) mode a
 * missing value takes the fill value and joins the ordinary comparison.
 *
 * Rows may number up to 2^31-1 (Methods, "Support for Big Data"); the row
 * index is 64-bit here anyway. An individual of length < 1 or with a column
 * outside [0, cols) is invalid: matched = negative = -1, its mask words 0.
 *
 * Mask layout: bit (r mod 64) of word (r / 64) in row i of an
 * [n_ind][ceil(rows/64)] uint64 array; bits past `rows` are 0.
 *
 * Plain loops over individuals x rows x columns in the order above; the
 * column loop stops once both P and N are false (a short-circuited AND).
 * Built without fast-math, so comparisons are IEEE-754 ordered compares
 * (NaN is unordered, -0 == +0, denormals are ordinary values).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_NAN_INCLUDE 1u
#define ORACLE_NEG_TRENDS  2u

#define ORACLE_OK      0
#define ORACLE_EINVAL -1

static int oracle_missing(float v, float sentinel)
{
    /* NaN, or equal (IEEE ==) to the sentinel; a NaN sentinel matches nothing. */
    return isnan(v) || v == sentinel;
}

int64_t ebic_oracle_mask_words(int64_t rows) { return (rows + 63) / 64; }

/*
 * X: row-major, rows x cols, row stride ld (>= cols) in elements.
 * offsets: n_ind + 1 int32; colidx: offsets[n_ind] int32.
 * matched, negative: n_ind int32 (negative may be NULL).
 * mmask, nmask: n_ind * ceil(rows/64) uint64 (either may be NULL).
 * threads: OpenMP threads over individuals (<= 0: library default).
 */
int ebic_oracle_eval(const float *X, int64_t rows, int32_t cols, int64_t ld,
                     const int32_t *offsets, const int32_t *colidx, int32_t n_ind,
                     uint32_t flags, float sentinel, float fill,
                     int32_t *matched, int32_t *negative,
                     uint64_t *mmask, uint64_t *nmask, int32_t threads)
{
    if (!X || rows <= 0 || cols <= 0 || ld < cols || !offsets || !matched || n_ind < 0)
        return ORACLE_EINVAL;
    if (n_ind > 0 && !colidx && offsets[n_ind] > 0)
        return ORACLE_EINVAL;
    if (flags & ~(ORACLE_NAN_INCLUDE | ORACLE_NEG_TRENDS))
        return ORACLE_EINVAL;
    const int include = (flags & ORACLE_NAN_INCLUDE) != 0;
    const int neg_on = (flags & ORACLE_NEG_TRENDS) != 0;
    if (include && isnan(fill))
        return ORACLE_EINVAL;
    const int64_t words = ebic_oracle_mask_words(rows);

#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int32_t i = 0; i < n_ind; ++i) {
        const int32_t begin = offsets[i], end = offsets[i + 1];
        const int32_t k = end - begin;
        const int32_t *c = colidx + begin;
        uint64_t *mrow = mmask ? mmask + (int64_t)i * words : NULL;
        uint64_t *nrow = nmask ? nmask + (int64_t)i * words : NULL;
        if (mrow) memset(mrow, 0, (size_t)words * sizeof(uint64_t));
        if (nrow) memset(nrow, 0, (size_t)words * sizeof(uint64_t));

        int valid = k >= 1;
        for (int32_t j = 0; valid && j < k; ++j)
            if (c[j] < 0 || c[j] >= cols) valid = 0;
        if (!valid) {
            matched[i] = -1;
            if (negative) negative[i] = -1;
            continue;
        }

        int64_t n_matched = 0, n_negative = 0;
        for (int64_t r = 0; r < rows; ++r) {
            const float *row = X + r * ld;
            int counted = 1;           /* cleared by a missing value in exclude mode */
            int pos = 1;               /* P so far */
            int neg = neg_on;          /* N so far */

            float prev = row[c[0]];
            if (oracle_missing(prev, sentinel)) {
                if (include) prev = fill;
                else counted = 0;
            }
            for (int32_t j = 1; counted && (pos || neg) && j < k; ++j) {
                float v = row[c[j]];
                if (oracle_missing(v, sentinel)) {
                    if (include) v = fill;
                    else { counted = 0; break; }
                }
                if (!(v >= prev)) pos = 0;
                if (!(v <= prev)) neg = 0;
                prev = v;
            }
            const int m_bit = counted && (pos || neg);
            const int n_bit = counted && neg && !pos;
            n_matched += m_bit;
            n_negative += n_bit;
            if (mrow && m_bit) mrow[r >> 6] |= (uint64_t)1 << (r & 63);
            if (nrow && n_bit) nrow[r >> 6] |= (uint64_t)1 << (r & 63);
        }
        matched[i] = (int32_t)n_matched;
        if (negative) negative[i] = (int32_t)n_negative;
    }
    return ORACLE_OK;
}

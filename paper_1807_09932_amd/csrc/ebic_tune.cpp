// ebic_tune.cpp -- launch-shape selection: defaults, the per-context tuning
// table, its JSON cache file, the forced-shape override, and the autotuner
// (ebic_autotune), which times candidate shapes on a sample and keeps the
// fastest per shape class.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_internal.h"
#include "ebic_runtime_internal.h"

namespace ebic {

static int32_t log2_bucket(int64_t v)
{
    int32_t b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

TuneKey tune_key(int64_t rows, int32_t cols, int32_t n, int64_t nnz)
{
    const int64_t kmean = (nnz > 0 && n > 0) ? (nnz + n - 1) / n : 0;
    return TuneKey{0, log2_bucket(rows), log2_bucket(cols), log2_bucket(n), log2_bucket(kmean)};
}

static TuneKey batch_key(int64_t total_ind, int64_t mean_rows, int32_t max_cols)
{
    return TuneKey{1, log2_bucket(mean_rows), log2_bucket(max_cols), log2_bucket(total_ind), 0};
}

// Defaults measured on MI355X: for the 436,444 x 64 workload the byte rank
// codes (four 64-row sub-tiles per lane word, two words per chunk) up to
// 128 columns, sixteen waves per block, groups of 200 individuals; for
// 129..512 columns (the 436,444 x 310 workload) the 10-bit codes, three
// sub-tiles per lane word, groups of 400. A request without codes for its
// mode falls back at launch.
static int32_t default_L(int32_t cols) { return cols <= 64 ? 4 : (cols <= 128 ? 2 : 1); }

LaunchCfg default_cfg(int64_t rows, int32_t cols, int32_t n)
{
    // The pairwise order bitmaps up to 512 columns (cols / 32 times the
    // FP32 matrix's bytes, built on first use): four waves per block, the
    // individuals per wave chosen at planning (P = 0).
    if (cols <= kDefaultPairCols) {
        LaunchCfg c;
        c.L = 1;
        c.W = 4;
        c.P = 0;
        c.staging = STAGE_PAIRS;
        c.blocks = 0;
        return c;
    }
    return default_codes_cfg(rows, cols, n);
}

LaunchCfg default_codes_cfg(int64_t rows, int32_t cols, int32_t n)
{
    (void)rows;
    LaunchCfg c;
    c.W = 16;
    c.P = std::max(1, std::min(n, 400));
    c.L = default_L(cols);
    c.staging = STAGE_LDS;
    if (cols <= kMaxByteCols) {
        // Two 256-row groups of byte codes per chunk, groups of 200.
        c.staging = STAGE_BYTES;
        c.L = 8;
        c.P = std::max(1, std::min(n, 200));
    } else if (cols <= kMaxT10Cols) {
        // 10-bit rank codes, one lane word of three rows per 192-row chunk
        // (cols x 256 bytes: two blocks per CU up to about 310 columns).
        c.staging = STAGE_T10;
        c.L = 3;
        c.P = std::max(1, std::min(n, 400));
    }
    c.blocks = 0;
    return c;
}

LaunchCfg default_batch_cfg(int32_t max_cols)
{
    // The pair bitmaps (as for one population) for the requests whose
    // matrices take them; the others get the rank codes' shape at planning.
    (void)max_cols;
    LaunchCfg c;
    c.L = 1;
    c.W = 4;
    c.P = 0;
    c.staging = STAGE_PAIRS;
    c.blocks = 0;
    return c;
}

LaunchCfg default_batch_codes_cfg(int32_t max_cols)
{
    LaunchCfg c;
    c.W = 16;
    c.P = 400;
    c.L = default_L(max_cols);
    c.staging = STAGE_LDS;
    if (max_cols <= kMaxByteCols) {
        c.staging = STAGE_BYTES;
        c.L = 4;
    } else if (max_cols <= kMaxT10Cols) {
        c.staging = STAGE_T10;  // one lane word of three rows, large groups
        c.L = 2;                // (the FP16 codes' sub-tiles, for requests without 10-bit codes)
        c.P = 1024;
    }
    c.blocks = 0;
    return c;
}

LaunchCfg tuned_cfg(ebic_ctx *ctx, int64_t rows, int32_t cols, int32_t n, int64_t nnz)
{
    if (nnz >= 0) {
        auto it = ctx->tuned.find(tune_key(rows, cols, n, nnz));
        if (it != ctx->tuned.end()) return it->second;
    }
    // Mean length unknown on the host (it lives in device memory): any entry
    // of the same rows/cols/population class will do.
    const TuneKey k = tune_key(rows, cols, n, 0);
    for (auto &kv : ctx->tuned)
        if (kv.first.kind == 0 && kv.first.rows_b == k.rows_b && kv.first.cols_b == k.cols_b &&
            kv.first.n_b == k.n_b)
            return kv.second;
    return default_cfg(rows, cols, n);
}

LaunchCfg tuned_batch_cfg(ebic_ctx *ctx, int64_t total_ind, int64_t mean_rows, int32_t max_cols,
                          int64_t nnz)
{
    (void)nnz;
    auto it = ctx->tuned.find(batch_key(total_ind, mean_rows, max_cols));
    if (it != ctx->tuned.end()) return it->second;
    return default_batch_cfg(max_cols);
}

// Minimal reader of the cache written by save_tune_cache: one JSON object
// per entry with integer fields.
static bool read_int(const std::string &obj, const char *key, int32_t *out)
{
    const std::string pat = std::string("\"") + key + "\"";
    size_t p = obj.find(pat);
    if (p == std::string::npos) return false;
    p = obj.find(':', p);
    if (p == std::string::npos) return false;
    long v = 0;
    if (std::sscanf(obj.c_str() + p + 1, " %ld", &v) != 1) return false;
    *out = (int32_t)v;
    return true;
}

static void read_cache(std::map<TuneKey, LaunchCfg> &out, const std::string &path)
{
    std::ifstream f(path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = s.find("\"entries\"");
    if (pos == std::string::npos) return;
    while (true) {
        size_t a = s.find('{', pos);
        if (a == std::string::npos) break;
        size_t b = s.find('}', a);
        if (b == std::string::npos) break;
        const std::string obj = s.substr(a, b - a + 1);
        pos = b + 1;
        TuneKey k{};
        LaunchCfg c;
        if (read_int(obj, "kind", &k.kind) && read_int(obj, "rows_b", &k.rows_b) &&
            read_int(obj, "cols_b", &k.cols_b) && read_int(obj, "n_b", &k.n_b) &&
            read_int(obj, "k_b", &k.k_b) && read_int(obj, "L", &c.L) && read_int(obj, "W", &c.W) &&
            read_int(obj, "P", &c.P) && read_int(obj, "staging", &c.staging)) {
            // (the shapes ebic_set_launch_shape accepts; anything else in the
            // file is skipped)
            const bool L_ok = c.L == 1 || c.L == 2 || c.L == 3 || c.L == 4 || c.L == 6 || c.L == 8 || c.L == 16;
            const bool stg_ok = c.staging == STAGE_LDS || c.staging == STAGE_DIRECT || c.staging == STAGE_CODES ||
                                c.staging == STAGE_BYTES || c.staging == STAGE_HALVES || c.staging == STAGE_T10 ||
                                c.staging == STAGE_PAIRS;
            if ((k.kind == 0 || k.kind == 1) && L_ok && c.W >= 1 && c.W <= 16 && c.P >= 1 && stg_ok) out[k] = c;
        }
    }
}

void load_tune_cache(ebic_ctx *ctx, const std::string &path) { read_cache(ctx->tuned, path); }

static void save_tune_cache(ebic_ctx *ctx, const std::string &path)
{
    // Merge: entries already in the file stay unless re-tuned here.
    std::map<TuneKey, LaunchCfg> merged;
    read_cache(merged, path);
    for (auto &kv : ctx->tuned) merged[kv.first] = kv.second;
    const std::string tmp_path = path + ".tmp";
    FILE *f = std::fopen(tmp_path.c_str(), "w");
    if (!f) fail(EBIC_EINVAL, "cannot write " + tmp_path);
    std::fprintf(f, "{\"arch\": \"%s\", \"entries\": [\n", ctx->arch.c_str());
    size_t i = 0;
    for (auto &kv : merged) {
        std::fprintf(f,
                     "  {\"kind\": %d, \"rows_b\": %d, \"cols_b\": %d, \"n_b\": %d, \"k_b\": %d, "
                     "\"L\": %d, \"W\": %d, \"P\": %d, \"staging\": %d}%s\n",
                     kv.first.kind, kv.first.rows_b, kv.first.cols_b, kv.first.n_b, kv.first.k_b,
                     kv.second.L, kv.second.W, kv.second.P, kv.second.staging,
                     ++i < merged.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
    if (std::rename(tmp_path.c_str(), path.c_str()) != 0) fail(EBIC_EINVAL, "cannot write " + path);
}

// Median of `reps` timed runs of `fn` (after one warm-up), in ms.
template <typename F>
static float time_ms(F &&fn, int reps, hipStream_t s)
{
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    std::vector<float> t;
    bool ok = true;
    for (int i = 0; i < reps + 1 && ok; ++i) {
        (void)hipEventRecord(e0, s);
        ok = fn();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (i > 0) t.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok || t.empty()) return INFINITY;
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

// The autotuner's final choice: the three fastest shapes of the first pass
// (median of three runs each) timed again in interleaved rounds (one run of
// each per round, nine rounds), so that clock drift and run-to-run noise
// fall on all of them alike; the lowest median wins. Shapes within a few
// percent of each other (as the byte kernel's 512- and 1024-row chunks
// are) would otherwise swap from one tuning to the next.
template <class Set, class F>
static LaunchCfg settle(std::vector<std::pair<float, LaunchCfg>> &timed, Set &&set_override, F &&fn,
                        hipStream_t s)
{
    if (timed.empty()) return LaunchCfg{};
    std::stable_sort(timed.begin(), timed.end(),
                     [](const std::pair<float, LaunchCfg> &a, const std::pair<float, LaunchCfg> &b) {
                         return a.first < b.first;
                     });
    const size_t k = std::min<size_t>(3, timed.size());
    if (k == 1) return timed[0].second;
    std::vector<std::vector<float>> t(k);
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    for (int round = 0; round < 9; ++round) {
        for (size_t i = 0; i < k; ++i) {
            set_override(timed[i].second);
            (void)hipEventRecord(e0, s);
            const bool ok = fn();
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = INFINITY;
            if (ok) (void)hipEventElapsedTime(&ms, e0, e1);
            t[i].push_back(ms);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    size_t best = 0;
    float best_ms = INFINITY;
    for (size_t i = 0; i < k; ++i) {
        std::sort(t[i].begin(), t[i].end());
        const float med = t[i][t[i].size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best = i;
        }
    }
    return timed[best].second;
}

}  // namespace ebic

using namespace ebic;

extern "C" {

ebic_status ebic_set_launch_shape(ebic_ctx *ctx, int32_t tiles_per_wave, int32_t waves_per_block,
                                  int32_t individuals_per_group, int32_t staging, int32_t blocks)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (waves_per_block == 0) {
            ctx->override_cfg = LaunchCfg();
            return;
        }
        if (!(tiles_per_wave == 1 || tiles_per_wave == 2 || tiles_per_wave == 3 || tiles_per_wave == 4 ||
              tiles_per_wave == 6 || tiles_per_wave == 8 || tiles_per_wave == 16) ||
            waves_per_block < 1 || waves_per_block > 16 ||
            (individuals_per_group < 1 && !(individuals_per_group == 0 && staging == STAGE_PAIRS)) ||
            !(staging == STAGE_LDS || staging == STAGE_DIRECT || staging == STAGE_CODES ||
              staging == STAGE_BYTES || staging == STAGE_HALVES || staging == STAGE_T10 ||
              staging == STAGE_PAIRS) ||
            blocks < 0)
            fail(EBIC_EINVAL, "launch shape out of range");
        LaunchCfg c;
        c.L = tiles_per_wave;
        c.W = waves_per_block;
        c.P = individuals_per_group;
        c.staging = staging;
        c.blocks = blocks;
        ctx->override_cfg = c;
    });
}

ebic_status ebic_autotune(ebic_ctx *ctx, const ebic_request *sample, int32_t n_reqs,
                          const char *cache_path)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if (n_reqs < 0 || (n_reqs > 0 && !sample)) fail(EBIC_EINVAL, "bad request array");
        DeviceGuard dg(ctx->device);
        hipStream_t s = nullptr;
        hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        LaunchCfg saved;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            saved = ctx->override_cfg;
        }
        auto set_override = [&](const LaunchCfg &c) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->override_cfg = c;
        };
        try {
            // One population at a time: one entry per distinct shape class.
            std::set<TuneKey> done;
            for (int32_t q = 0; q < n_reqs; ++q) {
                const ebic_request &r = sample[q];
                if (r.n_ind <= 0) continue;
                int32_t ends[2] = {0, 0};
                hip_check(hipMemcpy(&ends[0], r.d_offsets, sizeof(int32_t), hipMemcpyDeviceToHost),
                          "hipMemcpy");
                hip_check(hipMemcpy(&ends[1], r.d_offsets + r.n_ind, sizeof(int32_t),
                                    hipMemcpyDeviceToHost),
                          "hipMemcpy");
                int64_t rows;
                int32_t cols;
                bool have_codes, have_bytes, have_halves, have_t10;
                {
                    std::lock_guard<std::mutex> lk(ctx->mu);
                    const Matrix &m = ctx_matrix(ctx, r.matrix);
                    rows = m.dev.rows;
                    cols = m.dev.cols;
                    have_codes = ((r.flags & EBIC_NAN_INCLUDE) ? m.dev.Cfill : m.dev.C) != nullptr;
                    have_bytes = m.dev.B && ((r.flags & EBIC_NAN_INCLUDE) || m.dev.b_exclude);
                    have_halves = m.dev.Hc && ((r.flags & EBIC_NAN_INCLUDE) || m.dev.h_exclude);
                    have_t10 = m.dev.T10 && ((r.flags & EBIC_NAN_INCLUDE) || m.dev.t_exclude);
                }
                const TuneKey key = tune_key(rows, cols, r.n_ind, (int64_t)ends[1] - ends[0]);
                if (!done.insert(key).second) continue;
                auto eval_once = [&] {
                    return ebic_eval_population(ctx, r.matrix, r.n_ind, r.d_offsets, r.d_cols, r.flags,
                                                r.d_matched, r.d_negative, r.d_matched_mask, r.d_negative_mask,
                                                s) == EBIC_OK;
                };
                std::vector<std::pair<float, LaunchCfg>> timed;
                // The pairwise order bitmaps (built by the first of these
                // evaluations where they fit): waves per block and
                // individuals per wave, one chunk per block.
                if (cols <= kDefaultPairCols)
                    for (int W : {2, 4, 8})
                        for (int per_wave : {1, 2, 4, 8, 16}) {
                            LaunchCfg c;
                            c.L = 1;
                            c.W = W;
                            c.P = std::min(per_wave * W, r.n_ind);
                            c.staging = STAGE_PAIRS;
                            c.blocks = 1;
                            set_override(c);
                            const float ms = time_ms(eval_once, 3, s);
                            if (std::isfinite(ms)) timed.emplace_back(ms, c);
                        }
                for (int L : {1, 2, 3, 4, 6, 8, 16})
                    for (int W : {4, 8, 16})
                        for (int P : {200, 400, 800, 1600})
                            for (int stg : {(int)STAGE_LDS, (int)STAGE_DIRECT, (int)STAGE_CODES,
                                            (int)STAGE_BYTES, (int)STAGE_HALVES, (int)STAGE_T10}) {
                                if ((L == 3 || L == 6) != (stg == STAGE_T10)) continue;  // 10-bit codes: 3 or 6
                                if (stg == STAGE_T10 && !have_t10) continue;
                                LaunchCfg c;
                                c.L = L;
                                c.W = W;
                                c.P = std::min(P, r.n_ind);
                                c.staging = stg;
                                if (stg != STAGE_DIRECT &&
                                    item_lds_bytes(L, cols, stg, c.P,
                                                   stg == STAGE_HALVES || stg == STAGE_T10) > ctx->lds_per_block)
                                    continue;
                                if (stg == STAGE_CODES && (L < 2 || !have_codes)) continue;
                                if (stg == STAGE_BYTES && (L < 4 || !have_bytes)) continue;
                                if (L >= 8 && stg != STAGE_BYTES) continue;  // eight or 16 sub-tiles: byte codes only
                                if (L == 16 && (r.d_matched_mask || r.d_negative_mask)) continue;  // (counts only)
                                if (stg == STAGE_HALVES && ((L != 2 && L != 4) || !have_halves)) continue;
                                set_override(c);
                                const float ms = time_ms(eval_once, 3, s);
                                if (std::isfinite(ms)) timed.emplace_back(ms, c);
                            }
                LaunchCfg best = settle(timed, set_override, eval_once, s);
                if (best.W > 0) {
                    best.blocks = 0;  // re-derived from occupancy at launch (pairs: one chunk per run)
                    std::lock_guard<std::mutex> lk(ctx->mu);
                    ctx->tuned[key] = best;
                }
            }
            // The whole sample as one batch: tile width, waves and
            // individuals per work item for its shape class.
            if (n_reqs > 1) {
                int64_t total = 0, rows_sum = 0;
                int32_t max_cols = 1, live = 0;
                for (int32_t q = 0; q < n_reqs; ++q) {
                    if (sample[q].n_ind <= 0) continue;
                    std::lock_guard<std::mutex> lk(ctx->mu);
                    const Matrix &m = ctx_matrix(ctx, sample[q].matrix);
                    total += sample[q].n_ind;
                    rows_sum += m.dev.rows;
                    max_cols = std::max(max_cols, m.dev.cols);
                    ++live;
                }
                if (live > 0) {
                    const TuneKey key = batch_key(total, rows_sum / live, max_cols);
                    std::vector<std::pair<float, LaunchCfg>> timed;
                    auto batch_once = [&] { return ebic_eval_batch(ctx, sample, n_reqs, s) == EBIC_OK; };
                    if (max_cols <= kDefaultPairCols)
                        for (int W : {2, 4, 8})
                            for (int per_wave : {1, 2, 4, 8, 16}) {
                                LaunchCfg c;
                                c.L = 1;
                                c.W = W;
                                c.P = per_wave * W;
                                c.staging = STAGE_PAIRS;
                                set_override(c);
                                const float ms = time_ms(batch_once, 3, s);
                                if (std::isfinite(ms)) timed.emplace_back(ms, c);
                            }
                    for (int L : {1, 2, 4})
                        for (int W : {4, 8, 16})
                            for (int P : {128, 256, 512, 1024})
                                for (int stg : {(int)STAGE_LDS, (int)STAGE_CODES, (int)STAGE_BYTES,
                                                (int)STAGE_HALVES, (int)STAGE_T10}) {
                                if (stg == STAGE_CODES && L < 2) continue;
                                // (SWAR codes take their own sub-tiles in batches)
                                if ((stg == STAGE_BYTES || stg == STAGE_HALVES || stg == STAGE_T10) && L != 2) continue;
                                LaunchCfg c;
                                c.L = L;
                                c.W = W;
                                c.P = P;
                                c.staging = stg;
                                set_override(c);
                                const float ms = time_ms(batch_once, 3, s);
                                if (std::isfinite(ms)) timed.emplace_back(ms, c);
                            }
                    LaunchCfg best = settle(timed, set_override, batch_once, s);
                    if (best.W > 0) {
                        best.blocks = 0;
                        std::lock_guard<std::mutex> lk(ctx->mu);
                        ctx->tuned[key] = best;
                    }
                }
            }
        } catch (...) {
            set_override(saved);
            throw;
        }
        set_override(saved);
        if (cache_path && *cache_path) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            save_tune_cache(ctx, cache_path);
        }
    });
}

}  // extern "C"

// ebic_tune.cpp -- launch-shape selection: defaults, the per-context tuning
// table, its JSON cache file, and the autotuner (ebic_autotune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
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
    return TuneKey{log2_bucket(rows), log2_bucket(cols), log2_bucket(n), log2_bucket(kmean)};
}

LaunchCfg default_cfg(int64_t rows, int32_t cols, int32_t n)
{
    (void)rows;
    LaunchCfg c;
    c.W = 8;
    c.P = std::max(1, std::min(n, 1024));
    c.L = cols <= 96 ? 2 : 1;
    c.staging = STAGE_LDS;
    c.blocks = 0;
    return c;
}

LaunchCfg tuned_cfg(ebic_ctx *ctx, int64_t rows, int32_t cols, int32_t n, int64_t nnz)
{
    if (nnz >= 0) {
        auto it = ctx->tuned.find(tune_key(rows, cols, n, nnz));
        if (it != ctx->tuned.end()) return it->second;
    } else {
        // Population length unknown on the host: any entry of the same
        // rows/cols/n class will do.
        const TuneKey k = tune_key(rows, cols, n, 0);
        for (auto &kv : ctx->tuned)
            if (kv.first.rows_b == k.rows_b && kv.first.cols_b == k.cols_b && kv.first.n_b == k.n_b)
                return kv.second;
    }
    return default_cfg(rows, cols, n);
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

void load_tune_cache(ebic_ctx *ctx, const std::string &path)
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
        if (read_int(obj, "rows_b", &k.rows_b) && read_int(obj, "cols_b", &k.cols_b) &&
            read_int(obj, "n_b", &k.n_b) && read_int(obj, "k_b", &k.k_b) &&
            read_int(obj, "L", &c.L) && read_int(obj, "W", &c.W) && read_int(obj, "P", &c.P) &&
            read_int(obj, "staging", &c.staging)) {
            if ((c.L == 1 || c.L == 2 || c.L == 4) && c.W >= 1 && c.W <= 16 && c.P >= 1 &&
                (c.staging == STAGE_LDS || c.staging == STAGE_DIRECT))
                ctx->tuned[k] = c;
        }
    }
}

static void save_tune_cache(ebic_ctx *ctx, const std::string &path)
{
    // Merge: entries already in the file keep their place unless re-tuned.
    std::map<TuneKey, LaunchCfg> merged;
    {
        ebic_ctx tmp;
        load_tune_cache(&tmp, path);
        merged = tmp.tuned;
    }
    for (auto &kv : ctx->tuned) merged[kv.first] = kv.second;
    const std::string tmp_path = path + ".tmp";
    FILE *f = std::fopen(tmp_path.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\"arch\": \"%s\", \"entries\": [\n", ctx->arch.c_str());
    size_t i = 0;
    for (auto &kv : merged) {
        std::fprintf(f,
                     "  {\"rows_b\": %d, \"cols_b\": %d, \"n_b\": %d, \"k_b\": %d, \"L\": %d, "
                     "\"W\": %d, \"P\": %d, \"staging\": %d}%s\n",
                     kv.first.rows_b, kv.first.cols_b, kv.first.n_b, kv.first.k_b, kv.second.L,
                     kv.second.W, kv.second.P, kv.second.staging, ++i < merged.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
    std::rename(tmp_path.c_str(), path.c_str());
}

}  // namespace ebic

using namespace ebic;

namespace {
thread_local std::string t_err;
}

extern "C" {

ebic_status ebic_set_launch_shape(ebic_ctx *ctx, int32_t tiles_per_wave, int32_t waves_per_block,
                                  int32_t individuals_per_group, int32_t staging, int32_t blocks)
{
    if (!ctx) return EBIC_EINVAL;
    if (waves_per_block == 0) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->override_cfg = LaunchCfg();
        return EBIC_OK;
    }
    if (!(tiles_per_wave == 1 || tiles_per_wave == 2 || tiles_per_wave == 4) || waves_per_block < 1 ||
        waves_per_block > 16 || individuals_per_group < 1 ||
        !(staging == STAGE_LDS || staging == STAGE_DIRECT) || blocks < 0)
        return EBIC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    LaunchCfg c;
    c.L = tiles_per_wave;
    c.W = waves_per_block;
    c.P = individuals_per_group;
    c.staging = staging;
    c.blocks = blocks;
    ctx->override_cfg = c;
    return EBIC_OK;
}

}  // extern "C"

namespace ebic {

// Time one request under one launch shape: median of `reps` runs, in ms.
static float time_request(ebic_ctx *ctx, const ebic_request &r, const LaunchCfg &cfg, int reps,
                          hipStream_t s)
{
    const Matrix &m = ctx_matrix(ctx, r.matrix);
    EvalArgs a;
    a.m = m.dev;
    a.offsets = r.d_offsets;
    a.cols = r.d_cols;
    a.n = r.n_ind;
    a.flags = r.flags;
    a.matched = r.d_matched;
    a.negative = r.d_negative;
    a.mmask = r.d_matched_mask;
    a.nmask = r.d_negative_mask;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return INFINITY;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return INFINITY;
    }
    std::vector<float> t;
    for (int i = 0; i < reps + 1; ++i) {
        (void)hipEventRecord(e0, s);
        if (launch_eval(a, cfg, s) != hipSuccess) {
            (void)hipGetLastError();
            t.clear();
            break;
        }
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (i > 0) t.push_back(ms);  // the first run is a warm-up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (t.empty()) return INFINITY;
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace ebic

extern "C" ebic_status ebic_autotune(ebic_ctx *ctx, const ebic_request *sample, int32_t n_reqs,
                                     const char *cache_path)
{
    if (!ctx || (!sample && n_reqs > 0) || n_reqs < 0) return EBIC_EINVAL;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    hipStream_t s = nullptr;
    ebic_status st = EBIC_OK;
    try {
        for (int32_t q = 0; q < n_reqs; ++q) {
            const ebic_request &r = sample[q];
            if (r.n_ind <= 0) continue;
            // The host knows the population's size only through d_offsets.
            int32_t nnz = 0;
            if (hipMemcpy(&nnz, r.d_offsets + r.n_ind, sizeof(int32_t), hipMemcpyDeviceToHost) !=
                hipSuccess)
                return EBIC_EHIP;
            int32_t first = 0;
            (void)hipMemcpy(&first, r.d_offsets, sizeof(int32_t), hipMemcpyDeviceToHost);
            std::lock_guard<std::mutex> lk(ctx->mu);
            const Matrix &m = ctx_matrix(ctx, r.matrix);
            const TuneKey key = tune_key(m.dev.rows, m.dev.cols, r.n_ind, (int64_t)nnz - first);
            LaunchCfg best;
            float best_ms = INFINITY;
            for (int L : {1, 2, 4})
                for (int W : {4, 8, 16})
                    for (int P : {256, 1024, 4096})
                        for (int stg : {(int)STAGE_LDS, (int)STAGE_DIRECT}) {
                            LaunchCfg c;
                            c.L = L;
                            c.W = W;
                            c.P = std::min(P, r.n_ind);
                            c.staging = stg;
                            if (stg == STAGE_LDS && eval_lds_bytes(c, m.dev.cols) > ctx->lds_per_block)
                                continue;
                            if (eval_lds_bytes(c, m.dev.cols) > ctx->lds_per_block) continue;
                            int occ = eval_occupancy(c, m.dev.cols, r.flags);
                            if (occ <= 0) continue;
                            const int64_t n_tiles = (m.dev.rows + 63) / 64;
                            const int32_t groups = (r.n_ind + c.P - 1) / c.P;
                            int64_t bx = std::max<int64_t>(1, (int64_t)ctx->cu_count * occ / groups);
                            bx = std::min<int64_t>(bx, (n_tiles + L - 1) / L);
                            c.blocks = (int32_t)bx;
                            const float ms = time_request(ctx, r, c, 3, s);
                            if (ms < best_ms) {
                                best_ms = ms;
                                best = c;
                            }
                        }
            if (best.W > 0) {
                best.blocks = 0;  // re-derived from occupancy at launch
                ctx->tuned[key] = best;
            }
        }
        if (cache_path && *cache_path) save_tune_cache(ctx, cache_path);
    } catch (...) {
        st = EBIC_EINVAL;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    return st;
}

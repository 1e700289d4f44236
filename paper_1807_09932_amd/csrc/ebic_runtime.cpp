// ebic_runtime.cpp -- the C ABI declared in include/ebic.h: contexts, the
// resident-matrix registry, argument validation, launch planning and error
// reporting. Kernels live in ebic_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_internal.h"
#include "ebic_runtime_internal.h"

using namespace ebic;

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace ebic {

int log_level()
{
    static const int level = [] {
        const char *v = std::getenv("EBIC_LOG");
        return v && *v ? std::max(0, std::min(3, std::atoi(v))) : 0;
    }();
    return level;
}

void log_msg(int level, const std::string &msg)
{
    if (level > log_level()) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    std::fprintf(stderr, "[ebic] %s\n", msg.c_str());
    std::fflush(stderr);
}

void set_last_error(const std::string &msg)
{
    g_last_error = msg;
    if (!msg.empty()) log_msg(1, "error: " + msg);
}

FaultPlan parse_fault_plan(const char *spec)
{
    FaultPlan f;
    if (!spec) return f;
    std::string s(spec);
    size_t at = 0;
    while (at <= s.size()) {
        const size_t end = std::min(s.find(',', at), s.size());
        const std::string item = s.substr(at, end - at);
        const size_t colon = item.find(':');
        const std::string kind = item.substr(0, colon);
        int64_t n = 0;
        if (colon != std::string::npos) n = std::max<int64_t>(0, std::atoll(item.c_str() + colon + 1));
        if (kind == "alloc") f.alloc_after = n;
        else if (kind == "launch") f.launch_after = n;
        at = end + 1;
    }
    return f;
}

void fault_point_launch(ebic_ctx *ctx, const char *what)
{
    bool fire = false;
    {
        std::lock_guard<std::mutex> lk(ctx->fault_mu);
        if (ctx->fault.launch_after >= 0) {
            if (ctx->launches_done == ctx->fault.launch_after) {
                fire = true;
                ctx->fault.launch_after = -1;
            } else {
                ++ctx->launches_done;
            }
        }
    }
    if (fire) fail(EBIC_EHIP, std::string(what) + ": injected launch failure (EBIC_FAULT)");
}

void matrix_ref_locked(ebic_ctx *ctx, int32_t id)
{
    auto it = ctx->matrices.find(id);
    if (it == ctx->matrices.end()) fail(EBIC_ENOENT, "unknown matrix handle " + std::to_string(id));
    ++it->second.refs;
}

void matrix_unref(ebic_ctx *ctx, int32_t id)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->matrices.find(id);
    if (it != ctx->matrices.end() && it->second.refs > 0) --it->second.refs;
}

}  // namespace ebic

// ---------------------------------------------------------------------------
// Context helpers (also used by the batch and tuning code).
// ---------------------------------------------------------------------------
namespace ebic {

void *ctx_alloc(ebic_ctx *ctx, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    {
        std::lock_guard<std::mutex> lk(ctx->fault_mu);
        if (ctx->fault.alloc_after >= 0) {
            if (ctx->allocs_done == ctx->fault.alloc_after) {
                ctx->fault.alloc_after = -1;
                fail(EBIC_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                      " bytes: injected failure (EBIC_FAULT)");
            }
            ++ctx->allocs_done;
        }
    }
    void *p = nullptr;
    if (ctx->alloc) {
        p = ctx->alloc(bytes, ctx->alloc_user);
        if (!p) fail(EBIC_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {
            if (ctx->release) ctx->release(p, ctx->alloc_user);
            fail(EBIC_EINVAL, "allocator returned memory not aligned to 256 bytes");
        }
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(EBIC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                              hipGetErrorString(e));
    }
    return p;
}

void ctx_free(ebic_ctx *ctx, void *p)
{
    if (!p) return;
    if (ctx->alloc) {
        if (ctx->release) ctx->release(p, ctx->alloc_user);
        return;
    }
    (void)hipFree(p);
}

const Matrix &ctx_matrix(ebic_ctx *ctx, int32_t id)
{
    auto it = ctx->matrices.find(id);
    if (it == ctx->matrices.end()) fail(EBIC_ENOENT, "unknown matrix handle " + std::to_string(id));
    return it->second;
}

Matrix &ctx_matrix_mut(ebic_ctx *ctx, int32_t id)
{
    auto it = ctx->matrices.find(id);
    if (it == ctx->matrices.end()) fail(EBIC_ENOENT, "unknown matrix handle " + std::to_string(id));
    return it->second;
}

bool codes_buildable(const Matrix &m, bool include)
{
    return m.dev.cols <= kMaxCodeCols && (!include || m.Xfill != nullptr);
}

void build_fp16_codes(ebic_ctx *ctx, Matrix &m, bool include)
{
    if ((include ? m.Cfill : m.C) != nullptr) return;
    if (!codes_buildable(m, include)) fail(EBIC_EINVAL, "no rank codes can be built for this matrix and mode");
    DeviceGuard g(ctx->device);
    const size_t cbytes = (size_t)m.dev.ld * m.dev.cols * sizeof(uint16_t);
    uint16_t *C = static_cast<uint16_t *>(ctx_alloc(ctx, cbytes));
    hipStream_t s = nullptr;
    try {
        hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
        hip_check(launch_codes(include ? m.Xfill : m.X, m.dev.rows, m.dev.ld, m.dev.cols, C, s), "codes kernel");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        hip_check(hipStreamDestroy(s), "hipStreamDestroy");
        s = nullptr;
    } catch (...) {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        ctx_free(ctx, C);
        throw;
    }
    if (include) m.Cfill = C, m.dev.Cfill = C;
    else m.C = C, m.dev.C = C;
    m.bytes += cbytes;
    log_msg(2, std::string("built FP16 rank codes") + (include ? " of the fill copy" : "") + ": " +
                   std::to_string(cbytes) + " bytes");
}

bool halves_buildable(const Matrix &m, bool include)
{
    return m.dev.cols > kMaxByteCols && m.dev.cols <= kMaxCodeCols && (include || m.has_missing == 0);
}

void build_half_codes(ebic_ctx *ctx, Matrix &m)
{
    if (m.Hc) return;
    if (m.dev.cols <= kMaxByteCols || m.dev.cols > kMaxCodeCols)
        fail(EBIC_EINVAL, "16-bit rank codes serve matrices of 129 to 384 columns");
    DeviceGuard g(ctx->device);
    const int64_t rows = m.dev.rows;
    const int32_t cols = m.dev.cols;
    const int64_t rows_pad = (rows + 255) / 256 * 256;
    const int64_t ldh = rows_pad * 2;
    const size_t hbytes = (size_t)ldh * cols;
    const size_t tbytes = (size_t)((rows_pad + 511) / 512) * sizeof(int32_t);
    uint8_t *Hc = static_cast<uint8_t *>(ctx_alloc(ctx, hbytes + 256 + tbytes));
    int32_t *flag = reinterpret_cast<int32_t *>(Hc + hbytes);
    int32_t *ties = reinterpret_cast<int32_t *>(Hc + hbytes + 256);
    int32_t has_nan = 1;
    hipStream_t s = nullptr;
    try {
        hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
        hip_check(hipMemsetAsync(flag, 0, 256 + tbytes, s), "hipMemsetAsync");
        hip_check(launch_half_codes(m.X, rows, m.dev.ld, cols, m.dev.fill, Hc, ldh, flag, ties, s),
                  "16-bit codes kernel");
        hip_check(hipMemcpyAsync(&has_nan, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        hip_check(hipStreamDestroy(s), "hipStreamDestroy");
        s = nullptr;
    } catch (...) {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        ctx_free(ctx, Hc);
        throw;
    }
    m.Hc = Hc;
    m.dev.Hc = Hc;
    m.dev.Th = ties;
    m.dev.ldh = ldh;
    m.dev.h_exclude = has_nan == 0;
    m.bytes += hbytes + 256 + tbytes;
    log_msg(2, "built 16-bit rank codes: " + std::to_string(hbytes) + " bytes");
}

// The words of every pair, then each 2,048-row chunk's list of tied pairs.
static int64_t pairs_word_bytes(const Matrix &m)
{
    return (int64_t)m.dev.cols * m.dev.cols * pair_words(m.dev.rows) * (int64_t)sizeof(uint32_t);
}

static int64_t pairs_mark_bytes(const Matrix &m) { return pair_tie_bytes(m.dev.rows); }

static int64_t pairs_bytes(const Matrix &m) { return pairs_word_bytes(m) + pairs_mark_bytes(m); }

static const uint32_t *pairs_marks(const Matrix &m, const uint32_t *G)
{
    return G + pairs_word_bytes(m) / (int64_t)sizeof(uint32_t);
}

bool pairs_buildable(const Matrix &m)
{
    return m.dev.cols <= kMaxPairCols && m.dev.rows <= kMaxPairRows && pairs_bytes(m) <= kMaxPairBytes;
}

// The bitmaps a mode reads: exclude mode those of X; include mode those of
// the fill-substituted values, which are X's own when no cell is missing.
const uint32_t *pairs_for(const Matrix &m, bool include)
{
    if (!include) return m.Gx;
    if (m.has_missing == 0) return m.Gx;
    return m.Gf;
}

void build_pairs(ebic_ctx *ctx, Matrix &m, bool include)
{
    if (pairs_for(m, include)) return;
    if (!pairs_buildable(m))
        fail(EBIC_EINVAL, "pairwise order bitmaps serve matrices of at most " + std::to_string(kMaxPairCols) +
                              " columns, " + std::to_string(kMaxPairRows) + " rows and " +
                              std::to_string(kMaxPairBytes >> 30) + " GiB");
    const bool subst = include && m.has_missing != 0;  // (unknown counts as missing)
    DeviceGuard g(ctx->device);
    const int64_t w32 = pair_words(m.dev.rows);
    const size_t gbytes = (size_t)pairs_bytes(m);
    uint32_t *G = static_cast<uint32_t *>(ctx_alloc(ctx, gbytes));
    hipStream_t s = nullptr;
    try {
        hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
        uint32_t *F = const_cast<uint32_t *>(pairs_marks(m, G));
        hip_check(hipMemsetAsync(F, 0, (size_t)pairs_mark_bytes(m), s), "hipMemsetAsync");
        hip_check(launch_pair_bits(m.X, m.dev.rows, m.dev.ld, m.dev.cols, subst, m.dev.fill, G, w32, F, s),
                  "pair bitmaps kernel");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        hip_check(hipStreamDestroy(s), "hipStreamDestroy");
        s = nullptr;
    } catch (...) {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        ctx_free(ctx, G);
        throw;
    }
    if (subst) m.Gf = G, m.dev.Gf = G;
    else m.Gx = G, m.dev.Gx = G;
    m.dev.w32 = w32;
    m.bytes += gbytes;
    log_msg(2, std::string("built pairwise order bitmaps") + (subst ? " of the fill-substituted values" : "") +
                   ": " + std::to_string(gbytes) + " bytes");
}

// Launch shape for one population on one matrix.
LaunchCfg plan_eval(ebic_ctx *ctx, Matrix &m, int32_t n, int64_t nnz, uint32_t flags, CodesMode codes, bool masks)
{
    LaunchCfg cfg;
    if (ctx->override_cfg.W > 0) cfg = ctx->override_cfg;
    else cfg = tuned_cfg(ctx, m.dev.rows, m.dev.cols, n, nnz);
    const size_t lds_max = ctx->lds_per_block;
    const int32_t asked_P = cfg.P;  // (pairs: 0 = chosen here)
    cfg.P = std::max(1, std::min(cfg.P, std::max(1, n)));
    auto lds = [&](const LaunchCfg &c) { return item_lds_bytes(c.L, m.dev.cols, c.staging, c.P); };
    auto fits = [&](const LaunchCfg &c) { return lds(c) <= lds_max; };
    const bool include = (flags & EBIC_NAN_INCLUDE) != 0;
    // FP16 codes that are not resident count as available when they can be
    // built on first use; they are built below only if the plan stages them.
    const bool built_codes = (include ? m.dev.Cfill : m.dev.C) != nullptr;
    const bool have_codes = built_codes || (codes != CODES_EXISTING && codes_buildable(m, include));
    const bool have_bytes = m.dev.B && (include || m.dev.b_exclude);
    // (16-bit codes not built yet count as available where they can be
    // built; they are built below if the plan stages them)
    const bool have_halves = m.dev.Hc ? (include || m.dev.h_exclude)
                                      : codes != CODES_EXISTING && halves_buildable(m, include);
    const bool have_t10 = m.dev.T10 && (include || m.dev.t_exclude);
    // SWAR codes: bytes (up to 128 columns; one, two or four lane words per
    // row, L = 4, 8 or 16), 10-bit codes (up to 512 columns; one or two
    // words, L = 3 or 6) or
    // 16-bit codes (up to 384 columns; one or two words, L = 2 or 4). A
    // request without the kind its shape asks for takes another kind the
    // matrix has, else the FP16 codes (or the FP32 tile); a tile that does
    // not fit takes one word per row first.
    auto have_swar = [&](int32_t st) {
        return st == STAGE_BYTES ? have_bytes : st == STAGE_HALVES ? have_halves : st == STAGE_T10 ? have_t10 : false;
    };
    // Pairwise order bitmaps (built on first use where they fit): no tile,
    // one wave per individual and 2,048-row chunk.
    if (cfg.staging == STAGE_PAIRS) {
        bool have_pairs = pairs_for(m, include) != nullptr;
        if (!have_pairs && codes != CODES_EXISTING && pairs_buildable(m) && !m.pairs_failed) {
            have_pairs = true;  // (a report counts them as buildable)
            if (codes == CODES_BUILD) {
                try {
                    build_pairs(ctx, m, include);
                } catch (const Error &e) {
                    if (e.code != EBIC_ENOMEM) throw;
                    m.pairs_failed = true;
                    have_pairs = false;
                    log_msg(1, std::string("pair bitmaps not built (") + e.what() + "): rank codes instead");
                }
            }
        }
        if (have_pairs) {
            cfg.L = 1;
            cfg.cnt16 = false;
            if (asked_P <= 0) {
                // Individuals per wave: up to 8 where the chunks and
                // individuals give at least two waves per resident slot,
                // fewer (down to one) on smaller work.
                const int64_t chunks = pair_words(m.dev.rows) / 64;
                const int64_t slots = (int64_t)ctx->cu_count * 32;
                const int64_t per_wave = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)n * chunks / (2 * slots)));
                cfg.P = (int32_t)(per_wave * cfg.W);
            }
            cfg.P = std::max(1, std::min({cfg.P, 64 * cfg.W, std::max(1, n)}));
            cfg.blocks = (int32_t)(pair_words(m.dev.rows) / 64);  // (reported: the chunks)
            return cfg;
        }
        // without them: the shape planned for the rank codes
        cfg = default_codes_cfg(m.dev.rows, m.dev.cols, n);
        cfg.P = std::max(1, std::min(cfg.P, std::max(1, n)));
    }
    const bool asked_swar = cfg.staging == STAGE_BYTES || cfg.staging == STAGE_HALVES || cfg.staging == STAGE_T10;
    if (asked_swar && !have_swar(cfg.staging)) {
        const int32_t order[3] = {STAGE_BYTES, STAGE_T10, STAGE_HALVES};
        int32_t pick = -1;
        for (int32_t st : order)
            if (pick < 0 && have_swar(st)) pick = st;
        cfg.staging = pick >= 0 ? pick : (have_codes ? STAGE_CODES : STAGE_LDS);
    }
    // (four words per row group make counts only)
    if (cfg.staging == STAGE_BYTES) cfg.L = cfg.L >= 16 && !masks ? 16 : cfg.L >= 8 ? 8 : 4;
    if (cfg.staging == STAGE_BYTES && cfg.L == 16 && !fits(cfg)) cfg.L = 8;
    if (cfg.staging == STAGE_HALVES) cfg.L = cfg.L >= 4 ? 4 : 2;
    if (cfg.staging == STAGE_T10) cfg.L = cfg.L >= 6 ? 6 : 3;
    if (cfg.staging == STAGE_T10 && cfg.L == 6 && !fits(cfg)) cfg.L = 3;
    if (cfg.staging == STAGE_HALVES && cfg.L == 4 && !fits(cfg)) cfg.L = 2;
    if (cfg.staging == STAGE_BYTES && cfg.L == 8 && !fits(cfg)) cfg.L = 4;
    if ((cfg.staging == STAGE_HALVES || cfg.staging == STAGE_BYTES || cfg.staging == STAGE_T10) && !fits(cfg))
        cfg.staging = have_codes ? STAGE_CODES : STAGE_LDS;
    if (cfg.staging != STAGE_BYTES && cfg.staging != STAGE_T10) cfg.L = cfg.L == 3 ? 2 : std::min(cfg.L, 4);
    // Rank codes need codes for this mode and at least two sub-tiles.
    if (cfg.staging == STAGE_CODES && (!have_codes || cfg.L < 2)) cfg.staging = STAGE_LDS;
    // An FP32 tile that does not fit: the codes' tile (half the bytes) at the
    // same number of sub-tiles, if there are codes.
    if (cfg.staging == STAGE_LDS && !fits(cfg) && have_codes && cfg.L >= 2) {
        LaunchCfg c2 = cfg;
        c2.staging = STAGE_CODES;
        if (fits(c2)) cfg = c2;
    }
    // Then fewer rows per wave, FP32 staging, direct reads, until the shape fits.
    while (cfg.staging == STAGE_CODES && cfg.L > 2 && !fits(cfg)) cfg.L /= 2;
    if (cfg.staging == STAGE_CODES && !fits(cfg)) cfg.staging = STAGE_LDS;
    while (cfg.staging == STAGE_LDS && cfg.L > 1 && !fits(cfg)) cfg.L /= 2;
    if (cfg.staging == STAGE_LDS && !fits(cfg)) cfg.staging = STAGE_DIRECT;
    while (!fits(cfg) && cfg.P > 64) cfg.P /= 2;
    const int64_t n_tiles = (m.dev.rows + 63) / 64;
    const int32_t granule = cfg.staging == STAGE_BYTES && cfg.L == 16 ? 8 : cfg.L;  // (as the kernel cuts ranges)
    const int64_t n_chunks = (n_tiles + granule - 1) / granule;
    const int32_t groups = (n + cfg.P - 1) / cfg.P;
    const int32_t forced_blocks = cfg.blocks;
    auto derive_blocks = [&] {
        cfg.blocks = forced_blocks;
        if (cfg.blocks <= 0) {
            int occ = eval_occupancy(cfg, m.dev.cols, flags);
            if (occ <= 0) occ = 1;
            const int64_t slots = (int64_t)ctx->cu_count * occ;
            int64_t bx = std::max<int64_t>(1, slots / std::max(1, groups));
            bx = std::min<int64_t>(bx, n_chunks);
            cfg.blocks = (int32_t)std::max<int64_t>(1, bx);
        }
        cfg.blocks = (int32_t)std::min<int64_t>(cfg.blocks, std::max<int64_t>(1, n_tiles));
    };
    // With 16-bit codes the kernel keeps counts as 16-bit halves (half the
    // LDS beside a wide tile, which can leave room for a second block per
    // CU); that needs every block's tile range below 65,536 rows, so more
    // ranges are used where the matrix is taller.
    cfg.cnt16 = cfg.staging == STAGE_HALVES || cfg.staging == STAGE_T10;
    derive_blocks();
    if (cfg.cnt16) {
        const int64_t min_ranges = (n_chunks * cfg.L * 64 + 65535 - 1) / 65535;
        const int64_t need = std::max<int64_t>(min_ranges, 1);
        if ((n_chunks + cfg.blocks - 1) / cfg.blocks * cfg.L * 64 > 65535) {
            // the smallest range count whose largest range fits
            int64_t r = std::max<int64_t>(cfg.blocks, need);
            while ((n_chunks + r - 1) / r * cfg.L * 64 > 65535) ++r;
            cfg.blocks = (int32_t)std::min<int64_t>(r, std::max<int64_t>(1, n_tiles));
        }
    }
    if (cfg.staging == STAGE_CODES && !built_codes && codes == CODES_BUILD) build_fp16_codes(ctx, m, include);
    if (cfg.staging == STAGE_HALVES && !m.Hc && codes == CODES_BUILD) build_half_codes(ctx, m);
    return cfg;
}

ReqDesc make_desc(const Matrix &m, int32_t n, const int32_t *offsets, const int32_t *cols,
                  uint32_t flags, int32_t *matched, int32_t *negative, uint64_t *mmask,
                  uint64_t *nmask, int32_t staging)
{
    ReqDesc d{};
    const bool include = (flags & EBIC_NAN_INCLUDE) != 0;
    d.X = m.dev.X;
    d.C = nullptr;
    d.flags = flags & (kFlagInclude | kFlagNeg);
    if (staging == STAGE_CODES) {
        d.C = include ? m.dev.Cfill : m.dev.C;
        if (!d.C) fail(EBIC_EINVAL, "no rank codes for this matrix and mode");
        d.flags |= kFlagCodes;
    }
    d.B = nullptr;
    d.T = nullptr;
    d.ldb = m.dev.ldb;
    if (staging == STAGE_BYTES) {
        if (!m.dev.B || !(include || m.dev.b_exclude))
            fail(EBIC_EINVAL, "no byte rank codes for this matrix and mode");
        d.B = m.dev.B;
        d.T = m.dev.T;
        d.flags |= kFlagBytes;
    }
    if (staging == STAGE_HALVES) {
        if (!m.dev.Hc || !(include || m.dev.h_exclude))
            fail(EBIC_EINVAL, "no 16-bit rank codes for this matrix and mode");
        d.B = m.dev.Hc;
        d.T = m.dev.Th;
        d.ldb = m.dev.ldh;
        d.flags |= kFlagHalves;
    }
    if (staging == STAGE_T10) {
        if (!m.dev.T10 || !(include || m.dev.t_exclude))
            fail(EBIC_EINVAL, "no 10-bit rank codes for this matrix and mode");
        d.B = m.dev.T10;
        d.T = m.dev.Tt;
        d.ldb = m.dev.ld10;
        d.flags |= kFlagT10;
    }
    if (staging == STAGE_PAIRS) {
        const uint32_t *G = pairs_for(m, include);
        if (!G) fail(EBIC_EINVAL, "no pairwise order bitmaps for this matrix and mode");
        d.B = reinterpret_cast<const uint8_t *>(G);
        d.T = reinterpret_cast<const int32_t *>(pairs_marks(m, G));
        d.ldb = m.dev.w32;
        d.flags |= kFlagPairs;
    }
    if (staging == STAGE_DIRECT) {
        d.flags |= kFlagDirect;
        if (include) {
            if (m.dev.Xfill) d.X = m.dev.Xfill;
            else d.flags |= kFlagSubst;
        }
    }
    d.ld = m.dev.ld;
    d.rows = m.dev.rows;
    d.cols = m.dev.cols;
    d.fill = m.dev.fill;
    d.n = n;
    d.offsets = offsets;
    d.colidx = cols;
    d.matched = matched;
    d.negative = negative;
    d.mmask = mmask;
    d.nmask = nmask;
    d.head_base = 0;
    return d;
}

void upload_pinned(ebic_ctx *ctx, size_t bytes)
{
    // (called under ctx->mu)
    if (ctx->up_pin_bytes < bytes) {
        for (int b = 0; b < 2; ++b) {
            if (ctx->up_done[b]) hip_check(hipEventSynchronize(ctx->up_done[b]), "hipEventSynchronize");
            if (ctx->up_pin[b]) (void)hipHostFree(ctx->up_pin[b]);
            ctx->up_pin[b] = nullptr;
        }
        ctx->up_pin_bytes = 0;
        for (int b = 0; b < 2; ++b)
            hip_check(hipHostMalloc(&ctx->up_pin[b], bytes, hipHostMallocDefault), "hipHostMalloc");
        ctx->up_pin_bytes = bytes;
    }
    for (int b = 0; b < 2; ++b)
        if (!ctx->up_done[b])
            hip_check(hipEventCreateWithFlags(&ctx->up_done[b], hipEventDisableTiming), "hipEventCreate");
}

void pack_rows(const float *src, int64_t ld_src, bool col_major, int64_t r0, int64_t nr, int32_t cols, float *dst)
{
    // Row-major: rows r0 .. r0+nr of cols floats each -> dst[nr][cols].
    // Column-major: column c's entries r0 .. r0+nr -> dst[c][nr].
    const int64_t units = col_major ? cols : nr;
    const size_t unit_bytes = (size_t)(col_major ? nr : cols) * sizeof(float);
    const bool contiguous = col_major ? (ld_src == nr || cols == 1) : (ld_src == cols || nr == 1);
    const size_t total = (size_t)units * unit_bytes;
    unsigned nt = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    if (total < (4u << 20)) nt = 1;
    auto work = [&](unsigned t) {
        if (contiguous) {
            const char *from = reinterpret_cast<const char *>(col_major ? src + r0 : src + r0 * ld_src);
            const size_t lo = total * t / nt, hi = total * (t + 1) / nt;
            std::memcpy(reinterpret_cast<char *>(dst) + lo, from + lo, hi - lo);
            return;
        }
        const int64_t lo = units * t / nt, hi = units * (t + 1) / nt;
        for (int64_t u = lo; u < hi; ++u) {
            const float *from = col_major ? src + u * ld_src + r0 : src + (r0 + u) * ld_src;
            std::memcpy(reinterpret_cast<char *>(dst) + (size_t)u * unit_bytes, from, unit_bytes);
        }
    };
    if (nt == 1) {
        work(0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
}

void *stream_scratch(ebic_ctx *ctx, hipStream_t s, size_t bytes)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    Scratch &sc = ctx->scratch[s];
    if (sc.bytes >= bytes && sc.ptr) return sc.ptr;
    size_t want = std::max<size_t>(bytes, 64 << 10);
    want = std::max(want, sc.bytes * 2);
    if (sc.ptr) {
        // Work already enqueued on this stream may still read the old buffer.
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        ctx_free(ctx, sc.ptr);
        sc.ptr = nullptr;
        sc.bytes = 0;
    }
    sc.ptr = ctx_alloc(ctx, want);
    sc.bytes = want;
    return sc.ptr;
}

hipError_t ctx_launch_eval(ebic_ctx *ctx, const ReqDesc &d, const LaunchCfg &cfg, hipStream_t s)
{
    int32_t mode;
    unsigned long long *counter = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        mode = ctx->prof_mode;
        if (mode & 2) counter = ctx->d_step_counter;
    }
    IndHead *heads = static_cast<IndHead *>(stream_scratch(ctx, s, (size_t)d.n * sizeof(IndHead)));
    fault_point_launch(ctx, "evaluation launch");
    if (log_level() >= 3)
        log_msg(3, "eval n=" + std::to_string(d.n) + " rows=" + std::to_string(d.rows) + " cols=" +
                       std::to_string(d.cols) + " L=" + std::to_string(cfg.L) + " W=" + std::to_string(cfg.W) +
                       " P=" + std::to_string(cfg.P) + " staging=" + std::to_string(cfg.staging) +
                       " blocks=" + std::to_string(cfg.blocks));
    if (!(mode & 1)) return launch_eval(d, heads, cfg, counter, s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    e = launch_eval(d, heads, cfg, counter, s, e0, e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return e;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->prof_events.emplace_back(e0, e1);
    return hipSuccess;
}

}  // namespace ebic

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *ebic_last_error(void) { return g_last_error.c_str(); }

int64_t ebic_mask_words(int64_t rows) { return rows <= 0 ? 0 : (rows + 63) / 64; }

ebic_status ebic_create(int32_t hip_device, ebic_ctx **out)
{
    return guarded([&] {
        if (!out) fail(EBIC_EINVAL, "out is NULL");
        *out = nullptr;
        int n = 0;
        hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
        if (hip_device < 0 || hip_device >= n)
            fail(EBIC_EINVAL, "device " + std::to_string(hip_device) + " out of range (" +
                                  std::to_string(n) + " devices)");
        DeviceGuard g(hip_device);
        hip_check(noalloc_scratch_init(hip_device), "address of the no-allocation header buffer");
        hipDeviceProp_t prop;
        hip_check(hipGetDeviceProperties(&prop, hip_device), "hipGetDeviceProperties");
        auto *ctx = new ebic_ctx();
        ctx->device = hip_device;
        ctx->fault = parse_fault_plan(std::getenv("EBIC_FAULT"));
        ctx->cu_count = prop.multiProcessorCount;
        ctx->lds_per_block = std::max<size_t>(prop.sharedMemPerBlock, 65536);
        ctx->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
        ctx->arch = prop.gcnArchName;
        const char *cache = std::getenv("EBIC_TUNE_CACHE");
        if (cache && *cache) load_tune_cache(ctx, cache);
        *out = ctx;
    });
}

ebic_status ebic_destroy(ebic_ctx *ctx)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        {
            DeviceGuard g(ctx->device);
            (void)hipDeviceSynchronize();
            std::lock_guard<std::mutex> lk(ctx->mu);
            for (auto &kv : ctx->matrices) {
                ctx_free(ctx, kv.second.X);
                ctx_free(ctx, kv.second.Xfill);
                ctx_free(ctx, kv.second.C);
                ctx_free(ctx, kv.second.Cfill);
                ctx_free(ctx, kv.second.B);
                ctx_free(ctx, kv.second.Hc);
                ctx_free(ctx, kv.second.T10);
                ctx_free(ctx, kv.second.Gx);
                ctx_free(ctx, kv.second.Gf);
            }
            ctx->matrices.clear();
            destroy_batch_state(ctx);
            for (auto &pr : ctx->prof_events) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
            ctx->prof_events.clear();
            ctx_free(ctx, ctx->d_step_counter);
            ctx->d_step_counter = nullptr;
            for (auto &kv : ctx->scratch) ctx_free(ctx, kv.second.ptr);
            ctx->scratch.clear();
            for (int b = 0; b < 2; ++b) {
                if (ctx->up_done[b]) (void)hipEventDestroy(ctx->up_done[b]);
                if (ctx->up_pin[b]) (void)hipHostFree(ctx->up_pin[b]);
                ctx->up_done[b] = nullptr;
                ctx->up_pin[b] = nullptr;
            }
        }
        delete ctx;
    });
}

ebic_status ebic_set_allocator(ebic_ctx *ctx, void *(*alloc)(size_t, void *),
                               void (*release)(void *, void *), void *user)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if ((alloc == nullptr) != (release == nullptr))
            fail(EBIC_EINVAL, "alloc and release must both be set or both be NULL");
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!ctx->matrices.empty() || ctx->batch_state_allocated || ctx->d_step_counter ||
            !ctx->scratch.empty())
            fail(EBIC_EBUSY, "allocator can only change while nothing is resident");
        ctx->alloc = alloc;
        ctx->release = release;
        ctx->alloc_user = user;
    });
}

ebic_status ebic_upload_matrix(ebic_ctx *ctx, const float *src, int64_t rows, int32_t cols,
                               int64_t ld_src, uint32_t flags, float missing_sentinel,
                               float missing_fill, void *hip_stream, int32_t *out_matrix)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if (!src) fail(EBIC_EINVAL, "src is NULL");
        if (!out_matrix) fail(EBIC_EINVAL, "out_matrix is NULL");
        if (rows <= 0 || rows > INT32_MAX) fail(EBIC_EINVAL, "rows must be in 1 .. 2^31-1");
        if (cols <= 0) fail(EBIC_EINVAL, "cols must be >= 1");
        const uint32_t known = EBIC_SRC_DEVICE | EBIC_SRC_COL_MAJOR | EBIC_KEEP_FILL_COPY;
        if (flags & ~known) fail(EBIC_EINVAL, "unknown upload flags");
        if (std::isnan(missing_fill)) fail(EBIC_EINVAL, "missing_fill must not be NaN");
        const bool col_major = flags & EBIC_SRC_COL_MAJOR;
        if (col_major ? ld_src < rows : ld_src < cols)
            fail(EBIC_EINVAL, "ld_src smaller than the source's inner dimension");
        const bool on_device = flags & EBIC_SRC_DEVICE;
        hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);

        const auto t_start = std::chrono::steady_clock::now();
        DeviceGuard g(ctx->device);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Matrix m;
        m.dev.rows = rows;
        m.dev.cols = cols;
        m.dev.ld = (rows + 63) / 64 * 64;
        m.dev.fill = missing_fill;
        m.sentinel = missing_sentinel;
        const size_t bytes = (size_t)m.dev.ld * cols * sizeof(float);
        m.X = static_cast<float *>(ctx_alloc(ctx, bytes));
        m.bytes = bytes;
        float *staging = nullptr;
        try {
            if (flags & EBIC_KEEP_FILL_COPY) {
                m.Xfill = static_cast<float *>(ctx_alloc(ctx, bytes));
                m.bytes += bytes;
            }
            m.value_bytes = m.bytes;
            // Rows are laid out chunk by chunk through a bounded device
            // staging buffer. A host source is first packed (by several
            // threads) into one of two pinned buffers, so each chunk crosses
            // as one 1-D copy and the packing of a chunk overlaps the copy
            // and layout of the previous one.
            const int64_t chunk_bytes = 64ll << 20;
            int64_t chunk = std::max<int64_t>(64, chunk_bytes / ((int64_t)cols * 4) / 64 * 64);
            chunk = std::min<int64_t>(chunk, (rows + 63) / 64 * 64);
            const size_t stage_bytes = (size_t)chunk * cols * 4;
            if (!on_device) {
                staging = static_cast<float *>(ctx_alloc(ctx, stage_bytes));
                upload_pinned(ctx, stage_bytes);
            }
            int64_t ci = 0;
            for (int64_t r0 = 0; r0 < rows; r0 += chunk, ++ci) {
                const int64_t nr = std::min<int64_t>(chunk, rows - r0);
                const float *dsrc;
                int64_t dld;
                if (on_device) {
                    dsrc = col_major ? src + r0 : src + r0 * ld_src;
                    dld = ld_src;
                } else {
                    const int b = (int)(ci & 1);
                    // The copy that last read this pinned buffer has completed.
                    hip_check(hipEventSynchronize(ctx->up_done[b]), "hipEventSynchronize");
                    float *pin = static_cast<float *>(ctx->up_pin[b]);
                    pack_rows(src, ld_src, col_major, r0, nr, cols, pin);
                    hip_check(hipMemcpyAsync(staging, pin, (size_t)nr * cols * 4, hipMemcpyHostToDevice, s),
                              "hipMemcpyAsync");
                    hip_check(hipEventRecord(ctx->up_done[b], s), "hipEventRecord");
                    dsrc = staging;
                    dld = col_major ? nr : cols;
                }
                // (the next chunk's copy into `staging` follows this kernel on the stream)
                hip_check(launch_layout(dsrc, dld, col_major, nr, cols, r0, m.X, m.dev.ld,
                                        missing_sentinel, m.Xfill, missing_fill, s),
                          "layout kernel");
            }
            if (!on_device) hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
            hip_check(launch_zero_pad(m.X, rows, m.dev.ld, cols, s), "zero-pad kernel");
            if (m.Xfill) hip_check(launch_zero_pad(m.Xfill, rows, m.dev.ld, cols, s), "zero-pad kernel");
            // Byte rank codes for matrices of at most 128 columns: four rows
            // per 32-bit word. They encode the fill-substituted values, so
            // exclude mode may use them only if no cell is missing.
            int32_t has_nan = 1;
            if (cols <= kMaxByteCols) {
                // whole 512-row units plus one: a chunk of four 256-row groups
                // may start at any multiple of 512 rows
                m.dev.ldb = ((rows + 511) / 512 + 1) * 512;
                // Layout: codes | missing flag (256 bytes) | tie flags.
                const size_t bbytes = (size_t)m.dev.ldb * cols;
                const size_t tbytes = (size_t)(m.dev.ldb / 512) * sizeof(int32_t);
                m.B = static_cast<uint8_t *>(ctx_alloc(ctx, bbytes + 256 + tbytes));
                m.bytes += bbytes + 256 + tbytes;
                int32_t *flag = reinterpret_cast<int32_t *>(m.B + bbytes);
                int32_t *ties = reinterpret_cast<int32_t *>(m.B + bbytes + 256);
                hip_check(hipMemsetAsync(flag, 0, 256 + tbytes, s), "hipMemsetAsync");
                hip_check(launch_byte_codes(m.X, rows, m.dev.ld, cols, missing_fill, m.B, m.dev.ldb, flag, ties,
                                            s),
                          "byte codes kernel");
                m.dev.T = ties;
                hip_check(hipMemcpyAsync(&has_nan, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s),
                          "hipMemcpyAsync");
            }
            // (16-bit codes, two rows per 32-bit word, are built on first use:
            // the 10-bit codes serve the same widths with three.)
            int32_t has_nan_h = 1;
            // 10-bit codes (three rows per 32-bit word) for 129..512 columns.
            int32_t has_nan_t = 1;
            if (cols > kMaxByteCols && cols <= kMaxT10Cols) {
                // an even number of 192-row groups: a chunk of two groups
                // starts on an even one (the padding group stays zero)
                const int64_t groups = (rows + 2 * kT10Rows - 1) / (2 * kT10Rows) * 2;
                m.dev.ld10 = groups * 256;
                const size_t tb = (size_t)m.dev.ld10 * cols;
                const size_t fbytes = (size_t)groups * sizeof(int32_t);
                m.T10 = static_cast<uint8_t *>(ctx_alloc(ctx, tb + 256 + fbytes));
                m.bytes += tb + 256 + fbytes;
                int32_t *flag = reinterpret_cast<int32_t *>(m.T10 + tb);
                int32_t *ties = reinterpret_cast<int32_t *>(m.T10 + tb + 256);
                hip_check(hipMemsetAsync(m.T10, 0, tb + 256 + fbytes, s), "hipMemsetAsync");
                hip_check(launch_t10_codes(m.X, rows, m.dev.ld, cols, missing_fill, m.T10, m.dev.ld10, flag, ties, s),
                          "10-bit codes kernel");
                hip_check(hipMemcpyAsync(&has_nan_t, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s),
                          "hipMemcpyAsync");
                m.dev.Tt = ties;
            }
            hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
            m.dev.b_exclude = m.B && has_nan == 0;
            m.dev.h_exclude = m.Hc && has_nan_h == 0;
            m.dev.t_exclude = m.T10 && has_nan_t == 0;
            if (m.B) m.has_missing = has_nan != 0;
            if (m.Hc) m.has_missing = has_nan_h != 0;
            if (m.T10) m.has_missing = has_nan_t != 0;
            // FP16 rank codes (half the bytes of a staged FP32 tile, missing
            // cells kept as NaN) serve exclude mode where the SWAR codes
            // cannot: on a matrix with missing cells. Other uses (a shape
            // that stages them, include mode's codes of the fill copy) build
            // them on first use.
            if (cols <= kMaxCodeCols && m.has_missing == 1) {
                const size_t cbytes = (size_t)m.dev.ld * cols * sizeof(uint16_t);
                m.C = static_cast<uint16_t *>(ctx_alloc(ctx, cbytes));
                m.bytes += cbytes;
                hip_check(launch_codes(m.X, rows, m.dev.ld, cols, m.C, s), "codes kernel");
                hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
            }
        } catch (...) {
            (void)hipStreamSynchronize(s);  // nothing in flight reads what is freed
            ctx_free(ctx, staging);
            ctx_free(ctx, m.X);
            ctx_free(ctx, m.Xfill);
            ctx_free(ctx, m.C);
            ctx_free(ctx, m.Cfill);
            ctx_free(ctx, m.B);
            ctx_free(ctx, m.Hc);
            ctx_free(ctx, m.T10);
            ctx_free(ctx, m.Gx);
            ctx_free(ctx, m.Gf);
            throw;
        }
        ctx_free(ctx, staging);
        m.dev.X = m.X;
        m.dev.Xfill = m.Xfill;
        m.dev.C = m.C;
        m.dev.Cfill = m.Cfill;
        m.dev.B = m.B;
        m.dev.Hc = m.Hc;
        m.dev.T10 = m.T10;
        m.upload_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        const int32_t id = ctx->next_matrix++;
        ctx->matrices[id] = m;
        *out_matrix = id;
        log_msg(2, "uploaded matrix " + std::to_string(id) + ": " + std::to_string(rows) + " x " +
                       std::to_string(cols) + ", " + std::to_string(m.bytes) + " device bytes, " +
                       std::to_string(m.upload_ms) + " ms");
    });
}

ebic_status ebic_matrix_get_stats(ebic_ctx *ctx, int32_t matrix, ebic_matrix_stats *out)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if (!out) fail(EBIC_EINVAL, "out is NULL");
        DeviceGuard g(ctx->device);
        std::lock_guard<std::mutex> lk(ctx->mu);
        const Matrix &m = ctx_matrix(ctx, matrix);
        ebic_matrix_stats st{};
        st.rows = m.dev.rows;
        st.cols = m.dev.cols;
        st.code_sets = (m.Xfill ? EBIC_SET_FILL_COPY : 0u) | (m.C ? EBIC_SET_FP16 : 0u) |
                       (m.Cfill ? EBIC_SET_FP16_FILL : 0u) | (m.B ? EBIC_SET_U8 : 0u) | (m.Hc ? EBIC_SET_U16 : 0u) |
                       (m.T10 ? EBIC_SET_U10 : 0u) | (m.Gx ? EBIC_SET_PAIRS : 0u) |
                       (m.Gf ? EBIC_SET_PAIRS_FILL : 0u);
        st.value_bytes = (int64_t)m.value_bytes;
        st.code_bytes = (int64_t)(m.bytes - m.value_bytes);
        st.has_missing = m.has_missing;
        st.upload_ms = m.upload_ms;
        // (the tie flags of the default SWAR codes: bytes, else 10-bit codes)
        const int32_t *ties = m.B ? m.dev.T : m.T10 ? m.dev.Tt : m.Hc ? m.dev.Th : nullptr;
        if (ties) {
            const int64_t rows_pad = m.B ? (m.dev.rows + 511) / 512 * 512 : (m.dev.rows + 255) / 256 * 256;
            const int64_t n = m.B || !m.T10 ? (rows_pad + 511) / 512 : (m.dev.rows + kT10Rows - 1) / kT10Rows;
            std::vector<int32_t> h((size_t)n);
            hip_check(hipMemcpy(h.data(), ties, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost), "hipMemcpy");
            st.swar_chunks = n;
            for (int32_t v : h) st.swar_tie_chunks += v != 0;
        }
        *out = st;
    });
}

ebic_status ebic_matrix_info(ebic_ctx *ctx, int32_t matrix, int64_t *rows, int32_t *cols,
                             int64_t *device_bytes)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        std::lock_guard<std::mutex> lk(ctx->mu);
        const Matrix &m = ctx_matrix(ctx, matrix);
        if (rows) *rows = m.dev.rows;
        if (cols) *cols = m.dev.cols;
        if (device_bytes) *device_bytes = (int64_t)m.bytes;
    });
}

ebic_status ebic_release_matrix(ebic_ctx *ctx, int32_t matrix)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        DeviceGuard g(ctx->device);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Matrix m = ctx_matrix(ctx, matrix);
        if (m.refs > 0)
            fail(EBIC_EBUSY, "matrix " + std::to_string(matrix) + " is in use (" + std::to_string(m.refs) +
                                 " calls or serving requests hold it)");
        hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        ctx_free(ctx, m.X);
        ctx_free(ctx, m.Xfill);
        ctx_free(ctx, m.C);
        ctx_free(ctx, m.Cfill);
        ctx_free(ctx, m.B);
        ctx_free(ctx, m.Hc);
        ctx_free(ctx, m.T10);
        ctx_free(ctx, m.Gx);
        ctx_free(ctx, m.Gf);
        ctx->matrices.erase(matrix);
        log_msg(2, "released matrix " + std::to_string(matrix));
    });
}

ebic_status ebic_eval_population(ebic_ctx *ctx, int32_t matrix, int32_t n_ind,
                                 const int32_t *d_offsets, const int32_t *d_cols, uint32_t flags,
                                 int32_t *d_matched, int32_t *d_negative,
                                 uint64_t *d_matched_mask, uint64_t *d_negative_mask,
                                 void *hip_stream)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if (n_ind < 0) fail(EBIC_EINVAL, "n_ind < 0");
        if (flags & ~(EBIC_NAN_INCLUDE | EBIC_NEG_TRENDS)) fail(EBIC_EINVAL, "unknown eval flags");
        ReqDesc d;
        LaunchCfg cfg;
        MatrixHold hold(ctx);  // until the kernels are enqueued
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            Matrix &m = ctx_matrix_mut(ctx, matrix);
            if (n_ind == 0) return;
            if (!d_offsets || !d_cols || !d_matched)
                fail(EBIC_EINVAL, "d_offsets, d_cols and d_matched are required");
            cfg = plan_eval(ctx, m, n_ind, -1, flags, CODES_BUILD, d_matched_mask || d_negative_mask);
            d = make_desc(m, n_ind, d_offsets, d_cols, flags, d_matched, d_negative, d_matched_mask,
                          d_negative_mask, cfg.staging);
            hold.add_locked(matrix);
        }
        DeviceGuard g(ctx->device);
        hip_check(ctx_launch_eval(ctx, d, cfg, reinterpret_cast<hipStream_t>(hip_stream)),
                  "evaluation launch");
    });
}

ebic_status ebic_eval_population_noalloc(ebic_ctx *ctx, int32_t matrix, int32_t n_ind,
                                         const int32_t *d_offsets, const int32_t *d_cols, uint32_t flags,
                                         int32_t *d_matched, int32_t *d_negative,
                                         uint64_t *d_matched_mask, uint64_t *d_negative_mask,
                                         void *hip_stream)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if (n_ind < 0) fail(EBIC_EINVAL, "n_ind < 0");
        if (n_ind > kNoAllocMaxInd)
            fail(EBIC_EINVAL, "n_ind = " + std::to_string(n_ind) + " exceeds the no-allocation limit of " +
                                  std::to_string(kNoAllocMaxInd) + " individuals");
        if (flags & ~(EBIC_NAN_INCLUDE | EBIC_NEG_TRENDS)) fail(EBIC_EINVAL, "unknown eval flags");
        ReqDesc d;
        LaunchCfg cfg;
        MatrixHold hold(ctx);  // until the kernels are enqueued
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            Matrix &m = ctx_matrix_mut(ctx, matrix);
            if (n_ind == 0) return;
            if (!d_offsets || !d_cols || !d_matched)
                fail(EBIC_EINVAL, "d_offsets, d_cols and d_matched are required");
            cfg = plan_eval(ctx, m, n_ind, -1, flags, CODES_EXISTING,  // (allocates nothing)
                            d_matched_mask || d_negative_mask);
            d = make_desc(m, n_ind, d_offsets, d_cols, flags, d_matched, d_negative, d_matched_mask,
                          d_negative_mask, cfg.staging);
            hold.add_locked(matrix);
        }
        DeviceGuard g(ctx->device);
        fault_point_launch(ctx, "evaluation launch");
        IndHead *heads = noalloc_scratch(ctx->device);
        if (!heads) fail(EBIC_EHIP, "the no-allocation header buffer is not set up on this device");
        hip_check(launch_eval(d, heads, cfg, nullptr, reinterpret_cast<hipStream_t>(hip_stream)),
                  "evaluation launch");
    });
}

ebic_status ebic_plan_shape(ebic_ctx *ctx, int32_t matrix, int32_t n_ind, int64_t nnz,
                            int32_t *tiles_per_wave, int32_t *waves_per_block,
                            int32_t *individuals_per_group, int32_t *staging, int32_t *blocks)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if (n_ind <= 0) fail(EBIC_EINVAL, "n_ind must be >= 1");
        DeviceGuard g(ctx->device);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Matrix &m = ctx_matrix_mut(ctx, matrix);
        const LaunchCfg c = plan_eval(ctx, m, n_ind, nnz, EBIC_NEG_TRENDS, CODES_REPORT);
        if (tiles_per_wave) *tiles_per_wave = c.L;
        if (waves_per_block) *waves_per_block = c.W;
        if (individuals_per_group) *individuals_per_group = c.P;
        if (staging) *staging = c.staging;
        if (blocks) *blocks = c.blocks;
    });
}

ebic_status ebic_set_profiling(ebic_ctx *ctx, int32_t mode)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if (mode & ~3) fail(EBIC_EINVAL, "unknown profiling mode");
        DeviceGuard g(ctx->device);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if ((mode & 2) && !ctx->d_step_counter) {
            ctx->d_step_counter = static_cast<unsigned long long *>(ctx_alloc(ctx, 256));
            hip_check(hipMemset(ctx->d_step_counter, 0, sizeof(unsigned long long)), "hipMemset");
        }
        ctx->prof_mode = mode;
    });
}

ebic_status ebic_read_profile(ebic_ctx *ctx, int64_t *launches, double *kernel_ms,
                              int64_t *executed_steps)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        DeviceGuard g(ctx->device);
        hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        std::lock_guard<std::mutex> lk(ctx->mu);
        double ms = 0;
        for (auto &pr : ctx->prof_events) {
            float t = 0;
            if (hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) ms += t;
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        if (launches) *launches = (int64_t)ctx->prof_events.size();
        if (kernel_ms) *kernel_ms = ms;
        ctx->prof_events.clear();
        unsigned long long steps = 0;
        if (ctx->d_step_counter) {
            hip_check(hipMemcpy(&steps, ctx->d_step_counter, sizeof(steps), hipMemcpyDeviceToHost),
                      "hipMemcpy");
            hip_check(hipMemset(ctx->d_step_counter, 0, sizeof(steps)), "hipMemset");
        }
        if (executed_steps) *executed_steps = (int64_t)steps;
    });
}

}  // extern "C"

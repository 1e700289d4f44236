// ebic_batch.cpp -- ebic_eval_batch: many populations (of uneven sizes, with
// individuals of uneven lengths, over one or several resident matrices) in
// one replay of a captured HIP graph.
//
// The host planner puts each request on the pair bitmaps where its matrix
// has them (or can: they are built here on first use), else on the tiled
// kernel's stagings. Tiled requests become work items (individual group x
// tile range), ordered largest first, which the persistent tiled kernel's
// blocks take from a device-side counter. Pair requests are grouped by the
// bitmap set they read (a segment); per XCD slice of 2,048-row chunks, the
// fixed-grid pairs kernel walks each segment's chunks in order, all of its
// groups on a chunk before the next, with a static stride (no counter). The
// planner writes a batch arena (header, request descriptors, prefix sums of
// individuals, the pair lists and segments, the tiled items) into pinned
// host memory. A graph captured once per (stream, launch shapes, capacity)
// copies the arena to the device, runs the prep kernel (validation, output
// initialisation, the individual headers of each request's kind, zeroing
// the work counter) and the kernels the batch needs. The arena's device
// address is fixed per graph, so one graph serves every batch that fits its
// capacity; only the copy size is updated per replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_internal.h"
#include "ebic_runtime_internal.h"

namespace ebic {

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Header, request descriptors, prefix sums of individuals, the pair lists
// and segments (requests on pair bitmaps), then the tiled items.
struct ArenaLayout {
    size_t hdr = 0, descs = 0, first = 0, pq = 0, segs = 0, seg_req = 0, seg_gstart = 0, items = 0, bytes = 0;
    ArenaLayout(int32_t n_req, int32_t n_items)
    {
        hdr = 0;
        descs = align256(sizeof(BatchHeader));
        first = align256(descs + sizeof(ReqDesc) * (size_t)n_req);
        pq = align256(first + sizeof(int64_t) * (size_t)(n_req + 1));
        segs = align256(pq + sizeof(PairQueues));
        seg_req = align256(segs + sizeof(PairSeg) * (size_t)n_req);
        seg_gstart = align256(seg_req + sizeof(int32_t) * (size_t)n_req);
        items = align256(seg_gstart + sizeof(int32_t) * (size_t)n_req);
        bytes = align256(items + sizeof(Item) * (size_t)n_items);
    }
};

// One captured graph with the buffers its nodes point at.
struct GraphEntry {
    int32_t cap_req = 0, cap_items = 0;
    int64_t cap_ind = 0;
    void *d_arena = nullptr;
    IndHead *d_heads = nullptr;
    void *h_arena[2] = {nullptr, nullptr};  // pinned, used alternately
    hipEvent_t done[2] = {nullptr, nullptr};
    int next = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy_node = nullptr;
    std::mutex mu;  // one replay at a time per graph (its pinned buffers alternate)
};

// (stream, L, W, P, tile bytes, grid, capacities, counting, kernel set,
// which kernels run: 1 the tiled one, 2 the pairs one; the pairs kernel's
// W, an unused field, and its grid; its group size travels in the arena)
using GraphKey = std::tuple<hipStream_t, int32_t, int32_t, int32_t, int64_t, int32_t, int32_t,
                            int32_t, int64_t, bool, int32_t, int32_t, int32_t, int32_t, int32_t>;

void check(hipError_t e, const char *what) { hip_check(e, what); }

}  // namespace

struct BatchState {
    std::map<GraphKey, std::unique_ptr<GraphEntry>> graphs;
};

static void free_entry(ebic_ctx *ctx, GraphEntry *g)
{
    for (int i = 0; i < 2; ++i) {
        if (g->done[i]) {
            (void)hipEventSynchronize(g->done[i]);
            (void)hipEventDestroy(g->done[i]);
        }
        if (g->h_arena[i]) (void)hipHostFree(g->h_arena[i]);
    }
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    ctx_free(ctx, g->d_arena);
    ctx_free(ctx, g->d_heads);
}

void destroy_batch_state(ebic_ctx *ctx)
{
    if (!ctx->batch) return;
    for (auto &kv : ctx->batch->graphs) free_entry(ctx, kv.second.get());
    ctx->batch->graphs.clear();
    delete ctx->batch;
    ctx->batch = nullptr;
    ctx->batch_state_allocated = false;
}

// Launch shape of a batch: tuned if the context holds an entry for its
// shape class, else a default.
static LaunchCfg batch_cfg(ebic_ctx *ctx, int64_t total_ind, int64_t mean_rows, int32_t max_cols,
                           int64_t nnz)
{
    if (ctx->override_cfg.W > 0) return ctx->override_cfg;
    LaunchCfg c = tuned_batch_cfg(ctx, total_ind, mean_rows, max_cols, nnz);
    return c;
}

struct Plan {
    LaunchCfg cfg;
    std::vector<ReqDesc> descs;
    std::vector<int64_t> first;
    std::vector<Item> items;
    std::vector<int32_t> stagings;  // per request
    int32_t set = kBatchSetAll;     // the kernel instance (kBatchSet*)
    size_t tile_bytes = 0;
    int64_t total_ind = 0;
    int32_t grid = 0;
    // Requests on the pair bitmaps: their kernel's shape and item lists.
    bool pairs_shape = false;   // the shape asks for the bitmaps
    int32_t pW = 4, pP = 0, pgrid = 0;
    PairQueues pq{};
    std::vector<PairSeg> segs;
    std::vector<int32_t> seg_req, seg_gstart;
    bool any_pairs() const { return !segs.empty(); }
};

static Plan plan_batch(ebic_ctx *ctx, const ebic_request *reqs, int32_t n_reqs, bool count, CodesMode codes)
{
    Plan p;
    p.first.push_back(0);
    int64_t rows_sum = 0, nnz_hint = 0;
    int32_t max_cols = 1;
    int32_t live = 0;
    for (int32_t q = 0; q < n_reqs; ++q) {
        const ebic_request &r = reqs[q];
        if (r.n_ind < 0) fail(EBIC_EINVAL, "request " + std::to_string(q) + ": n_ind < 0");
        if (r.flags & ~(EBIC_NAN_INCLUDE | EBIC_NEG_TRENDS))
            fail(EBIC_EINVAL, "request " + std::to_string(q) + ": unknown flags");
        const Matrix &m = ctx_matrix(ctx, r.matrix);
        if (r.n_ind > 0 && (!r.d_offsets || !r.d_cols || !r.d_matched))
            fail(EBIC_EINVAL, "request " + std::to_string(q) +
                                  ": d_offsets, d_cols and d_matched are required");
        if (r.n_ind > 0) {
            rows_sum += m.dev.rows;
            max_cols = std::max(max_cols, m.dev.cols);
            ++live;
        }
    }
    (void)nnz_hint;
    const int64_t mean_rows = live ? rows_sum / live : 1;
    int64_t total = 0;
    for (int32_t q = 0; q < n_reqs; ++q) total += std::max(0, reqs[q].n_ind);
    p.cfg = batch_cfg(ctx, total, mean_rows, max_cols, -1);
    // (the bitmaps up to 512 columns, or up to 1,024 under a forced shape)
    const int32_t pair_cols = ctx->override_cfg.W > 0 ? kMaxPairCols : kDefaultPairCols;
    if (p.cfg.staging == STAGE_PAIRS) {
        // The bitmaps' kernel takes this shape; requests that cannot read
        // bitmaps take the rank codes' default shape.
        p.pairs_shape = true;
        p.pW = std::max(1, std::min(16, p.cfg.W));
        p.pP = p.cfg.P;
        p.cfg = default_batch_codes_cfg(max_cols);
    }
    LaunchCfg &c = p.cfg;
    const size_t lds_max = ctx->lds_per_block - 256;  // room for the kernel's static LDS
    if (c.L == 8) c.L = 4;  // (batches stage at most four sub-tiles per chunk)
    if (c.L != 1 && c.L != 2 && c.L != 4) c.L = 2;
    c.W = std::max(1, std::min(16, c.W));
    c.P = std::max(1, c.P);

    // Staging per request. When the shape asks for SWAR codes, each request
    // takes the kind its matrix has for its mode, each at its own number of
    // sub-tiles: bytes (four), else the kind the shape names among the
    // 10-bit (three) and 16-bit (two) codes, else the other of the two. Then
    // the FP16 rank codes when the shape asks for codes (or the FP32 tile
    // does not fit) and they exist and fit; else the FP32 tile if it fits
    // next to the counts, else direct reads.
    std::vector<int32_t> tiles_of;  // sub-tiles per chunk, per request (0: on the pair bitmaps)
    for (int32_t q = 0; q < n_reqs; ++q) {
        const ebic_request &r = reqs[q];
        Matrix &m = ctx_matrix_mut(ctx, r.matrix);
        const bool include = (r.flags & EBIC_NAN_INCLUDE) != 0;
        if (p.pairs_shape && r.n_ind > 0 && m.dev.cols <= pair_cols) {
            // The pair bitmaps where they exist or can be built (a report
            // plans them unbuilt: its descriptors are never launched).
            bool have = pairs_for(m, include) != nullptr;
            if (!have && codes != CODES_EXISTING && pairs_buildable(m) && !m.pairs_failed) {
                have = true;
                if (codes == CODES_BUILD) {
                    try {
                        build_pairs(ctx, m, include);
                    } catch (const Error &e) {
                        if (e.code != EBIC_ENOMEM) throw;
                        m.pairs_failed = true;
                        have = false;
                        log_msg(1, std::string("pair bitmaps not built (") + e.what() + "): rank codes instead");
                    }
                }
            }
            if (have) {
                const bool built = pairs_for(m, include) != nullptr;
                ReqDesc d = make_desc(m, r.n_ind, r.d_offsets, r.d_cols, r.flags, r.d_matched, r.d_negative,
                                      r.d_matched_mask, r.d_negative_mask, built ? STAGE_PAIRS : STAGE_LDS);
                d.head_base = p.first.back();
                p.stagings.push_back(STAGE_PAIRS);
                tiles_of.push_back(0);
                p.descs.push_back(d);
                p.first.push_back(p.first.back() + d.n);
                continue;
            }
        }
        // FP16 codes not resident yet count as available when they can be
        // built; they are built below if this request stages them.
        const bool built_codes = (include ? m.dev.Cfill : m.dev.C) != nullptr;
        const bool have_codes = built_codes || (codes != CODES_EXISTING && codes_buildable(m, include));
        const bool have_bytes = m.dev.B && (include || m.dev.b_exclude);
        const bool have_halves = m.dev.Hc ? (include || m.dev.h_exclude)
                                          : codes != CODES_EXISTING && halves_buildable(m, include);
        const bool have_t10 = m.dev.T10 && (include || m.dev.t_exclude);
        auto fits = [&](int32_t stg) {
            return tile_lds_bytes(batch_tiles(stg, c.L), m.dev.cols, stg) + count_lds_bytes(c.P) <= lds_max;
        };
        int32_t staging = STAGE_DIRECT;
        const bool codes_ok = have_codes && c.L >= 2 && fits(STAGE_CODES);
        const bool wants_swar = c.staging == STAGE_BYTES || c.staging == STAGE_HALVES || c.staging == STAGE_T10;
        const bool wants_codes = c.staging == STAGE_CODES || wants_swar;
        const int32_t wide1 = c.staging == STAGE_HALVES ? STAGE_HALVES : STAGE_T10;
        const int32_t wide2 = wide1 == STAGE_HALVES ? STAGE_T10 : STAGE_HALVES;
        auto have = [&](int32_t stg) { return stg == STAGE_T10 ? have_t10 : have_halves; };
        if (wants_swar && have_bytes && fits(STAGE_BYTES)) staging = STAGE_BYTES;
        else if (wants_swar && have(wide1) && fits(wide1)) staging = wide1;
        else if (wants_swar && have(wide2) && fits(wide2)) staging = wide2;
        else if (codes_ok && (wants_codes || !fits(STAGE_LDS))) staging = STAGE_CODES;
        else if (fits(STAGE_LDS)) staging = STAGE_LDS;
        if (staging == STAGE_CODES && !built_codes && codes == CODES_BUILD && r.n_ind > 0)
            build_fp16_codes(ctx, m, include);
        if (staging == STAGE_HALVES && !m.Hc && codes == CODES_BUILD && r.n_ind > 0) build_half_codes(ctx, m);
        // (a report plans codes that are not built yet: its descriptors are
        // never launched)
        const bool unbuilt = (staging == STAGE_CODES && (include ? m.dev.Cfill : m.dev.C) == nullptr) ||
                             (staging == STAGE_HALVES && !m.dev.Hc);
        ReqDesc d = make_desc(m, std::max(0, r.n_ind), r.d_offsets, r.d_cols, r.flags, r.d_matched,
                              r.d_negative, r.d_matched_mask, r.d_negative_mask,
                              unbuilt && (codes == CODES_REPORT || r.n_ind <= 0) ? STAGE_LDS : staging);
        d.head_base = p.first.back();
        p.stagings.push_back(staging);
        tiles_of.push_back(batch_tiles(staging, c.L));
        p.tile_bytes = std::max(p.tile_bytes, tile_lds_bytes(tiles_of.back(), m.dev.cols, staging));
        p.descs.push_back(d);
        p.first.push_back(p.first.back() + d.n);
    }
    p.total_ind = p.first.back();
    // The kernel instance: one compiled for a single kind of SWAR codes when
    // every live request stages that kind.
    {
        int32_t used = 0;
        for (size_t q = 0; q < p.stagings.size(); ++q) {
            if (p.descs[q].n <= 0 || p.stagings[q] == STAGE_PAIRS) continue;
            const int32_t stg = p.stagings[q];
            used |= stg == STAGE_BYTES ? kBatchSetBytes
                    : stg == STAGE_HALVES ? kBatchSetHalves
                    : stg == STAGE_T10 ? kBatchSetT10
                    : stg == STAGE_CODES ? kBatchSetCodes : kBatchSetValues;
        }
        p.set = used == kBatchSetBytes || used == kBatchSetHalves || used == kBatchSetT10 ? used : kBatchSetAll;
    }

    const size_t lds = p.tile_bytes + count_lds_bytes(c.P);
    int occ = batch_occupancy(c.L, p.set, c.W, lds);
    if (occ <= 0) occ = 1;
    p.grid = c.blocks > 0 ? c.blocks : ctx->cu_count * occ;

    // Items: each request is cut into groups of <= P individuals and tile
    // ranges so that the whole batch has about 8 items per resident block,
    // in proportion to each request's work (individuals x tiles).
    double units = 0;
    for (int32_t q = 0; q < n_reqs; ++q)
        if (tiles_of[q] > 0) units += (double)p.descs[q].n * (double)((p.descs[q].rows + 63) / 64);
    const double target = 8.0 * p.grid;
    struct Est {
        Item it;
        double cost;
    };
    std::vector<Est> est;
    for (int32_t q = 0; q < n_reqs; ++q) {
        const ReqDesc &d = p.descs[q];
        if (d.n == 0 || tiles_of[q] == 0) continue;
        const int64_t tiles = (d.rows + 63) / 64;
        const int32_t Lq = tiles_of[q];
        const int64_t chunks = (tiles + Lq - 1) / Lq;  // ranges start on a multiple of Lq tiles
        const int32_t groups = (d.n + c.P - 1) / c.P;
        const double share = units > 0 ? target * (double)d.n * (double)tiles / units : 1.0;
        int64_t ranges = (int64_t)std::max(1.0, share / groups + 0.5);
        ranges = std::min<int64_t>(ranges, chunks);
        for (int32_t g = 0; g < groups; ++g) {
            const int32_t i0 = g * c.P;
            const int32_t np = std::min(c.P, d.n - i0);
            for (int64_t r = 0; r < ranges; ++r) {
                Item it{};
                it.req = q;
                it.i0 = i0;
                it.np = np;
                it.t0 = (int32_t)(r * chunks / ranges * Lq);
                it.t1 = (int32_t)std::min<int64_t>(tiles, (r + 1) * chunks / ranges * Lq);
                if (it.t1 <= it.t0) continue;
                est.push_back({it, (double)np * (double)(it.t1 - it.t0)});
            }
        }
    }
    std::stable_sort(est.begin(), est.end(), [](const Est &a, const Est &b) { return a.cost > b.cost; });
    p.items.reserve(est.size());
    for (auto &e : est) p.items.push_back(e.it);

    // The pair requests: segments by bitmap set (requests in order), groups
    // of pP individuals, and per XCD slice the items of each segment (its
    // chunks of that slice x its groups).
    {
        int64_t ind_chunks = 0;
        for (int32_t q = 0; q < n_reqs; ++q)
            if (p.stagings[q] == STAGE_PAIRS && p.descs[q].n > 0)
                ind_chunks += (int64_t)p.descs[q].n * ((p.descs[q].rows + 2047) / 2048);
        if (p.pairs_shape && ind_chunks > 0) {
            if (p.pP <= 0) {
                // individuals per wave: up to 8 where the work gives at least
                // two waves per resident slot, at least 2 (an item's lookup
                // costs about what one individual's chunk does)
                const int64_t slots = (int64_t)ctx->cu_count * 32;
                p.pP = (int32_t)(p.pW * std::max<int64_t>(2, std::min<int64_t>(8, ind_chunks / (2 * slots))));
            }
            p.pP = std::max(1, std::min(p.pP, 64 * p.pW));
            std::vector<const uint8_t *> keys;
            for (int32_t q = 0; q < n_reqs; ++q) {
                const ReqDesc &d = p.descs[q];
                if (p.stagings[q] != STAGE_PAIRS || d.n <= 0) continue;
                size_t g = 0;
                while (g < keys.size() && keys[g] != d.B) ++g;
                if (g == keys.size()) {
                    keys.push_back(d.B);
                    PairSeg sg{};
                    sg.n_chunks = (int32_t)((d.rows + 2047) / 2048);
                    p.segs.push_back(sg);
                }
            }
            // entries grouped by segment, requests in order within each
            for (size_t g = 0; g < keys.size(); ++g) {
                PairSeg &sg = p.segs[g];
                sg.e0 = (int32_t)p.seg_req.size();
                for (int32_t q = 0; q < n_reqs; ++q) {
                    const ReqDesc &d = p.descs[q];
                    if (p.stagings[q] != STAGE_PAIRS || d.n <= 0 || d.B != keys[g]) continue;
                    p.seg_req.push_back(q);
                    p.seg_gstart.push_back(sg.groups);
                    sg.groups += (d.n + p.pP - 1) / p.pP;
                    ++sg.n_req;
                }
            }
            for (int x = 0; x < 8; ++x) {
                int64_t k = 0;
                for (auto &sg : p.segs) {
                    sg.base[x] = (int32_t)k;
                    const int64_t in_slice = sg.n_chunks > x ? (sg.n_chunks - x + 7) / 8 : 0;
                    k += in_slice * sg.groups;
                }
                if (k > INT32_MAX) fail(EBIC_EINVAL, "batch too large for one launch");
                p.pq.total[x] = (int32_t)k;
            }
            p.pq.n_seg = (int32_t)p.segs.size();
            p.pq.P = p.pP;  // (in the arena: graphs do not depend on it)
            int occ = pairs_batch_occupancy(p.pW);
            if (occ <= 0) occ = 1;
            p.pgrid = std::max(8, ctx->cu_count * occ / 8 * 8);
        }
    }
    (void)count;
    return p;
}

struct GraphSpec {
    GraphKey key;
    int32_t cap_req, cap_items;
    int64_t cap_ind;
};

static GraphSpec graph_spec(hipStream_t s, const Plan &p, bool count)
{
    // Capacities rounded up to powers of two, with floors that cover typical
    // batches, so that batches of different sizes share a graph (a capture
    // costs milliseconds; the floors cost about 1.3 MB per graph).
    auto pow2 = [](int64_t x) {
        int64_t v = 1;
        while (v < x) v <<= 1;
        return v;
    };
    GraphSpec g;
    g.cap_req = (int32_t)pow2(std::max<int64_t>(64, (int64_t)p.descs.size()));
    g.cap_items = (int32_t)pow2(std::max<int64_t>(8192, (int64_t)p.items.size()));
    g.cap_ind = pow2(std::max<int64_t>(16384, p.total_ind));
    // (the shape of a kernel that does not run stays out of the key)
    const bool tiled = !p.items.empty(), pairs = p.any_pairs();
    const int32_t kernels = (tiled ? 1 : 0) | (pairs ? 2 : 0);
    g.key = GraphKey{s, tiled ? p.cfg.L : 0, tiled ? p.cfg.W : 0, tiled ? p.cfg.P : 0,
                     tiled ? (int64_t)p.tile_bytes : 0, tiled ? p.grid : 0, g.cap_req, g.cap_items, g.cap_ind,
                     count, tiled ? p.set : 0, kernels, pairs ? p.pW : 0, 0, pairs ? p.pgrid : 0};
    return g;
}

// Capture a new graph for `spec`. Holds no context lock: the capture runs on
// a stream of its own in relaxed capture mode, so evaluations, uploads and
// builds of codes or bitmaps on other threads and streams proceed meanwhile
// without being refused as unsafe during a capture.
static std::unique_ptr<GraphEntry> capture_graph(ebic_ctx *ctx, const GraphSpec &spec, const Plan &p,
                                                 bool count)
{
    auto g = std::make_unique<GraphEntry>();
    g->cap_req = spec.cap_req;
    g->cap_items = spec.cap_items;
    g->cap_ind = spec.cap_ind;
    const ArenaLayout lay(spec.cap_req, spec.cap_items);
    hipStream_t cs = nullptr;
    try {
        g->d_arena = ctx_alloc(ctx, lay.bytes);
        g->d_heads = static_cast<IndHead *>(ctx_alloc(ctx, (size_t)spec.cap_ind * sizeof(IndHead)));
        for (int i = 0; i < 2; ++i) {
            check(hipHostMalloc(&g->h_arena[i], lay.bytes, hipHostMallocDefault), "hipHostMalloc");
            std::memset(g->h_arena[i], 0, lay.bytes);
            check(hipEventCreateWithFlags(&g->done[i], hipEventDisableTiming), "hipEventCreate");
        }
        char *da = static_cast<char *>(g->d_arena);
        const int prep_blocks = std::max(1, ctx->cu_count * 8);  // four waves each, one individual per wave
        unsigned long long *counter = count ? ctx->d_step_counter : nullptr;
        check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
        check(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
        hipError_t e = hipMemcpyAsync(da, g->h_arena[0], lay.bytes, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess)
            e = launch_batch(reinterpret_cast<BatchHeader *>(da + lay.hdr),
                             reinterpret_cast<const ReqDesc *>(da + lay.descs),
                             reinterpret_cast<const int64_t *>(da + lay.first),
                             reinterpret_cast<const Item *>(da + lay.items), g->d_heads, p.cfg.L,
                             p.set, p.cfg.W, p.cfg.P, p.tile_bytes, p.items.empty() ? 0 : p.grid, prep_blocks,
                             counter, cs);
        if (e == hipSuccess && p.any_pairs())
            e = launch_pairs_batch(reinterpret_cast<const PairQueues *>(da + lay.pq),
                                   reinterpret_cast<const ReqDesc *>(da + lay.descs),
                                   reinterpret_cast<const PairSeg *>(da + lay.segs),
                                   reinterpret_cast<const int32_t *>(da + lay.seg_req),
                                   reinterpret_cast<const int32_t *>(da + lay.seg_gstart), g->d_heads, p.pW,
                                   p.pgrid, counter, cs);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        check(e, "batch capture");
        check(e2, "hipStreamEndCapture");
        g->graph = graph;
        check(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        size_t nn = 0;
        check(hipGraphGetNodes(graph, nullptr, &nn), "hipGraphGetNodes");
        std::vector<hipGraphNode_t> nodes(nn);
        check(hipGraphGetNodes(graph, nodes.data(), &nn), "hipGraphGetNodes");
        for (auto n : nodes) {
            hipGraphNodeType t;
            check(hipGraphNodeGetType(n, &t), "hipGraphNodeGetType");
            if (t == hipGraphNodeTypeMemcpy) g->copy_node = n;
        }
        if (!g->copy_node) fail(EBIC_EHIP, "captured batch graph has no copy node");
        check(hipStreamDestroy(cs), "hipStreamDestroy");
        cs = nullptr;
    } catch (...) {
        if (cs) (void)hipStreamDestroy(cs);
        free_entry(ctx, g.get());
        throw;
    }
    return g;
}

}  // namespace ebic

using namespace ebic;

extern "C" ebic_status ebic_plan_batch_shape(ebic_ctx *ctx, const ebic_request *reqs, int32_t n_reqs,
                                             int32_t *tiles_per_wave, int32_t *waves_per_block,
                                             int32_t *individuals_per_group, int32_t *stagings,
                                             int32_t *blocks)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if (n_reqs < 1 || !reqs) fail(EBIC_EINVAL, "need at least one request");
        DeviceGuard dg(ctx->device);
        std::lock_guard<std::mutex> lk(ctx->mu);
        const Plan p = plan_batch(ctx, reqs, n_reqs, false, CODES_REPORT);
        if (tiles_per_wave) *tiles_per_wave = p.cfg.L;
        if (waves_per_block) *waves_per_block = p.cfg.W;
        // (a batch with no request on the tiled kernel reports the pairs
        // kernel's shape)
        const bool pairs_only = p.items.empty() && p.any_pairs();
        if (tiles_per_wave && pairs_only) *tiles_per_wave = 1;
        if (waves_per_block && pairs_only) *waves_per_block = p.pW;
        if (individuals_per_group) *individuals_per_group = pairs_only ? p.pP : p.cfg.P;
        if (blocks) *blocks = pairs_only ? p.pgrid : p.grid;
        if (stagings)
            for (int32_t q = 0; q < n_reqs; ++q) stagings[q] = p.stagings[q];
    });
}

extern "C" ebic_status ebic_eval_batch(ebic_ctx *ctx, const ebic_request *reqs, int32_t n_reqs,
                                       void *hip_stream)
{
    return guarded([&] {
        if (!ctx) fail(EBIC_EINVAL, "ctx is NULL");
        if (n_reqs < 0 || (n_reqs > 0 && !reqs)) fail(EBIC_EINVAL, "bad request array");
        if (n_reqs == 0) return;
        hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
        DeviceGuard dg(ctx->device);
        Plan p;
        int32_t prof_mode;
        MatrixHold hold(ctx);  // until the graph is launched
        {
            std::lock_guard<std::mutex> lk2(ctx->mu);
            p = plan_batch(ctx, reqs, n_reqs, false, CODES_BUILD);
            prof_mode = ctx->prof_mode;
            for (int32_t q = 0; q < n_reqs; ++q)
                if (reqs[q].n_ind > 0) hold.add_locked(reqs[q].matrix);
        }
        if (p.items.empty() && !p.any_pairs()) return;  // every population is empty
        const bool count = (prof_mode & 2) != 0;
        const GraphSpec spec = graph_spec(s, p, count);
        GraphEntry *g = nullptr;
        {
            std::lock_guard<std::mutex> lk(ctx->batch_mu);
            if (!ctx->batch) {
                ctx->batch = new BatchState();
                ctx->batch_state_allocated = true;
            }
            auto it = ctx->batch->graphs.find(spec.key);
            if (it != ctx->batch->graphs.end()) g = it->second.get();
        }
        if (!g) {
            std::unique_ptr<GraphEntry> fresh = capture_graph(ctx, spec, p, count);
            std::lock_guard<std::mutex> lk(ctx->batch_mu);
            auto it = ctx->batch->graphs.find(spec.key);
            if (it != ctx->batch->graphs.end()) {  // another thread captured it meanwhile
                free_entry(ctx, fresh.get());
                g = it->second.get();
            } else {
                g = fresh.get();
                ctx->batch->graphs.emplace(spec.key, std::move(fresh));
                std::lock_guard<std::mutex> lk2(ctx->mu);
                ++ctx->graph_captures;
            }
        }
        fault_point_launch(ctx, "batch launch");
        std::lock_guard<std::mutex> lkg(g->mu);
        const int slot = g->next;
        g->next ^= 1;
        // This slot's pinned buffer was last read by the launch two calls ago.
        check(hipEventSynchronize(g->done[slot]), "hipEventSynchronize");
        const ArenaLayout cap(g->cap_req, g->cap_items);
        char *h = static_cast<char *>(g->h_arena[slot]);
        BatchHeader bh{};
        bh.n_req = (int32_t)p.descs.size();
        bh.n_items = (int32_t)p.items.size();
        bh.total_ind = p.total_ind;
        std::memcpy(h + cap.hdr, &bh, sizeof(bh));
        std::memcpy(h + cap.descs, p.descs.data(), sizeof(ReqDesc) * p.descs.size());
        std::memcpy(h + cap.first, p.first.data(), sizeof(int64_t) * p.first.size());
        std::memcpy(h + cap.pq, &p.pq, sizeof(PairQueues));
        if (!p.segs.empty()) {
            std::memcpy(h + cap.segs, p.segs.data(), sizeof(PairSeg) * p.segs.size());
            std::memcpy(h + cap.seg_req, p.seg_req.data(), sizeof(int32_t) * p.seg_req.size());
            std::memcpy(h + cap.seg_gstart, p.seg_gstart.data(), sizeof(int32_t) * p.seg_gstart.size());
        }
        std::memcpy(h + cap.items, p.items.data(), sizeof(Item) * p.items.size());
        const size_t used = cap.items + sizeof(Item) * p.items.size();
        check(hipGraphExecMemcpyNodeSetParams1D(g->exec, g->copy_node, g->d_arena, h, used,
                                                hipMemcpyHostToDevice),
              "hipGraphExecMemcpyNodeSetParams1D");
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof_mode & 1) {
            check(hipEventCreate(&e0), "hipEventCreate");
            check(hipEventCreate(&e1), "hipEventCreate");
            check(hipEventRecord(e0, s), "hipEventRecord");
        }
        check(hipGraphLaunch(g->exec, s), "hipGraphLaunch");
        if (prof_mode & 1) {
            check(hipEventRecord(e1, s), "hipEventRecord");
            std::lock_guard<std::mutex> lk2(ctx->mu);
            ctx->prof_events.emplace_back(e0, e1);
        }
        check(hipEventRecord(g->done[slot], s), "hipEventRecord");
    });
}

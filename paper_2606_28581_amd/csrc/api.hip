// C-ABI layer of the SatSplat gfx950 hot path: validation, the plan and its workspace,
// and the order in which the kernels of one call run on the caller's stream.
#include "satsplat.h"
#include "ss_internal.h"
#include "ss_mlp.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace ss;

namespace {

thread_local std::string g_err;

ss_status fail(ss_status code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define SS_HIP(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(SS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int bits_for(int64_t count)
{
    int b = 0;
    while (b < 32 && (int64_t(1) << b) < count) ++b;
    return b;
}

}  // namespace

struct ss_context {
    int device = 0;
    int cus = 0;
    std::string arch;
    char *scratch = nullptr;   // this device's address of the allocation-free MLP scratch
};

// Offsets (bytes) of every buffer inside the workspace.
struct Layout {
    size_t views_main, views_sun, suncam, counters, flags;
    size_t mk_a, mk_b, mv_a, mv_b, sorted_main;
    size_t sk_a, sk_b, sv_a, sv_b, sorted_sun;
    size_t rec_main, tiles_main, counts_main, offs_main, scanparts;
    size_t pk_a, pv_a, pk_b, pv_b, ranges_main, recgrad, colour_parts, dF_parts;
    size_t rec_sun, tiles_sun, counts_sun, offs_sun, qk_a, qv_a, qk_b, qv_b, ranges_sun;
    size_t sun_depth, bounds, radix_temp, tmask_sun, cmask, cmask_bytes, stat_main, stat_sun;
    size_t torder_main, torder_sun, torder_parts;
    size_t inv_order, vis_rank;
    size_t geom_seeds, geom_cams, geom_parts;
    size_t total;
};

// HIP-event stage timer (enabled by ss_plan_set_timing).
struct StageTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Pending { int stage; hipEvent_t a, b; };
    std::vector<Pending> pending;
    double ms[SS_NUM_STAGES] = {0};
    int64_t count[SS_NUM_STAGES] = {0};
    hipEvent_t take()
    {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    ~StageTimer()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

struct ss_plan {
    StageTimer timer;
    ss_context *ctx = nullptr;
    ss_raster_settings st{};
    int64_t n = 0;
    int32_t nv = 0;
    std::vector<int32_t> W, H;
    std::vector<ViewDesc> vmain, vsun;
    int32_t tiles_main = 0, tiles_sun = 0;          // for the current tile size
    int32_t tiles_main_max = 0, tiles_sun_max = 0;  // for the smallest tile size (8)
    int64_t P = 0;
    int64_t cap_main = 0, cap_sun = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Layout L{};
    bool fwd_valid = false, sun_valid = false;
    // bumped whenever the workspace or the settings change: a captured graph holds raw
    // pointers into the workspace and kernels specialised for the settings
    uint64_t generation = 1;
    uint32_t *order_main = nullptr, *order_sun = nullptr;
    bool sun_order_shared = false;   // the last shadow pass used the main-view order buffers
    uint32_t *lists_main = nullptr, *lists_sun = nullptr;
    // raster dispatch orders built with the current binning (null: static XCD order)
    const uint32_t *torder_main = nullptr, *torder_sun = nullptr;
    template <class T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

// Records an event pair around a stage when timing is on.
struct StageScope {
    ss_plan *p;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr;
    StageScope(ss_plan *p_, int stage_, hipStream_t st_) : p(p_), stage(stage_), st(st_)
    {
        if (p->timer.on && (a = p->timer.take()) != nullptr) (void)hipEventRecord(a, st);
    }
    ~StageScope()
    {
        if (!a) return;
        hipEvent_t b = p->timer.take();
        if (!b) return;
        (void)hipEventRecord(b, st);
        p->timer.pending.push_back({stage, a, b});
    }
};

static void build_views(ss_plan *p)
{
    const int ts = p->st.tile_size;
    const int S = p->st.sun_map_size;
    p->vmain.resize(p->nv);
    p->vsun.resize(p->nv);
    int64_t pix = 0;
    int32_t toff = 0, soff = 0;
    for (int v = 0; v < p->nv; ++v) {
        ViewDesc d{};
        d.W = p->W[v]; d.H = p->H[v];
        d.tiles_x = (d.W + ts - 1) / ts; d.tiles_y = (d.H + ts - 1) / ts;
        d.pix_off = pix; d.tile_off = toff;
        pix += (int64_t)d.W * d.H;
        toff += d.tiles_x * d.tiles_y;
        p->vmain[v] = d;
        ViewDesc s{};
        s.W = S; s.H = S;
        s.tiles_x = (S + ts - 1) / ts; s.tiles_y = s.tiles_x;
        s.pix_off = (int64_t)v * S * S; s.tile_off = soff;
        soff += s.tiles_x * s.tiles_y;
        p->vsun[v] = s;
    }
    p->P = pix;
    p->tiles_main = toff;
    p->tiles_sun = soff;
}

static void max_tiles(ss_plan *p)
{
    int64_t tm = 0, tsn = 0;
    const int S = p->st.sun_map_size;
    for (int v = 0; v < p->nv; ++v) {
        tm += (int64_t)((p->W[v] + 7) / 8) * ((p->H[v] + 7) / 8);
        tsn += (int64_t)((S + 7) / 8) * ((S + 7) / 8);
    }
    p->tiles_main_max = (int32_t)tm;
    p->tiles_sun_max = (int32_t)tsn;
}

static int64_t max_view_pixels(const ss_plan *p)
{
    int64_t m = 0;
    for (int v = 0; v < p->nv; ++v) m = std::max<int64_t>(m, (int64_t)p->W[v] * p->H[v]);
    return m;
}

static Layout make_layout(const ss_plan *p, int64_t cm, int64_t cs)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
    const size_t n = (size_t)p->n, nv = (size_t)p->nv, vn = n * nv;
    const size_t S = (size_t)p->st.sun_map_size;
    L.views_main = take(nv * sizeof(ViewDesc));
    L.views_sun = take(nv * sizeof(ViewDesc));
    L.suncam = take(nv * sizeof(SunCam));
    L.counters = take(16 * sizeof(unsigned long long));
    L.stat_main = take((size_t)kStatSlots * kStatStride * sizeof(unsigned long long));
    L.stat_sun = take((size_t)kStatSlots * kStatStride * sizeof(unsigned long long));
    L.flags = take(16 * sizeof(uint32_t));
    L.mk_a = take(n * 4); L.mk_b = take(n * 4); L.mv_a = take(n * 4); L.mv_b = take(n * 4);
    L.sorted_main = take(n * 16 * 4);
    L.sk_a = take(n * 4); L.sk_b = take(n * 4); L.sv_a = take(n * 4); L.sv_b = take(n * 4);
    L.sorted_sun = take(n * 16 * 4);
    L.rec_main = take(vn * kRecStride4 * 16);
    L.tiles_main = take(vn * sizeof(short4));
    L.counts_main = take(vn * 4);
    L.offs_main = take((vn + 1) * 4);
    L.scanparts = take(scan_temp_elems((int64_t)vn) * 4);
    L.pk_a = take((size_t)cm * 4); L.pv_a = take((size_t)cm * 4);
    L.pk_b = take((size_t)cm * 4); L.pv_b = take((size_t)cm * 4);
    L.ranges_main = take((size_t)p->tiles_main_max * 8);
    L.recgrad = take(vn * kGradFloats * 4);
    L.colour_parts = take((size_t)p->tiles_main_max * 16 * 4);
    L.dF_parts = take((size_t)project_bwd_blocks(p->n) * nv * 8 * 4);
    L.rec_sun = take(vn * kSunRecStride4 * 16);
    L.tiles_sun = take(vn * sizeof(short4));
    L.counts_sun = take(vn * 4);
    L.offs_sun = take((vn + 1) * 4);
    L.qk_a = take((size_t)cs * 4); L.qv_a = take((size_t)cs * 4);
    L.qk_b = take((size_t)cs * 4); L.qv_b = take((size_t)cs * 4);
    L.ranges_sun = take((size_t)p->tiles_sun_max * 8);
    L.sun_depth = take(nv * S * S * 4);
    L.bounds = take((size_t)bounds_blocks(p->n) * 6 * 8);
    L.radix_temp = take(radix_temp_bytes(std::max<int64_t>(p->n, std::max(cm, cs)), p->nv));
    L.tmask_sun = take((size_t)p->tiles_sun_max * 4);
    L.inv_order = take(n * 4);
    L.vis_rank = take(vn * 4);
    // forward -> backward contributor masks of 8x8 tiles (other sizes use the box test)
    L.cmask_bytes = p->st.tile_size == 8 ? cmask_words(cm, p->tiles_main_max) * 8 : 0;
    L.cmask = take(L.cmask_bytes);
    // heavy-first raster dispatch orders and their per-XCD block counts
    L.torder_main = take((size_t)p->tiles_main_max * 4);
    L.torder_sun = take((size_t)p->tiles_sun_max * 4);
    L.torder_parts = take(((size_t)8 * tile_order_blocks(std::max(p->tiles_main_max, p->tiles_sun_max)) + 8) * 4);
    // normal-consistency loss: per-pixel depth-adjoint seeds, per-view cameras, block sums
    L.geom_seeds = take((size_t)p->P * 8);
    L.geom_cams = take(nv * sizeof(GeomCam));
    L.geom_parts = take((size_t)std::max(normal_loss_blocks(p->vmain.data(), p->nv) * 10,
                                         l1_blocks(max_view_pixels(p))) * nv * 8);
    L.total = o;
    return L;
}

static ss_status check_settings(const ss_raster_settings *s)
{
    if (!s) return fail(SS_ERR_INVALID_ARG, "settings is NULL");
    if (s->struct_size != sizeof(ss_raster_settings))
        return fail(SS_ERR_INVALID_ARG, "settings.struct_size mismatch");
    if (s->tile_size != 8 && s->tile_size != 16 && s->tile_size != 32)
        return fail(SS_ERR_UNSUPPORTED, "tile_size must be 8, 16 or 32");
    if (s->batch_depth < 1 || s->batch_depth > 256)
        return fail(SS_ERR_UNSUPPORTED, "batch_depth must be in [1, 256]");
    if (!(s->alpha_min > 0.f && s->alpha_min < 1.f) || !(s->alpha_max >= s->alpha_min) ||
        !(s->alpha_max < 1.f) || !(s->T_min > 0.f && s->T_min < 1.f) ||
        !(s->lowpass_sigma > 0.f) || !(s->det_rel_eps >= 0.f) ||
        (s->lowpass_mode != 0 && s->lowpass_mode != 1) || !(s->esm_c > 0.f))
        return fail(SS_ERR_INVALID_ARG, "threshold setting out of range");
    if (s->sun_map_size < 8 || s->sun_map_size > 16384)
        return fail(SS_ERR_INVALID_ARG, "sun_map_size must be in [8, 16384]");
    if (s->tile_order != 0 && s->tile_order != 1)
        return fail(SS_ERR_INVALID_ARG, "tile_order must be 0 or 1");
    return SS_OK;
}

static RasterConsts consts(const ss_raster_settings &s)
{
    RasterConsts rc{};
    rc.alpha_min = s.alpha_min;
    rc.alpha_max = s.alpha_max;
    rc.T_min = s.T_min;
    const double sig = (double)s.lowpass_sigma;
    rc.inv_s2 = (float)(1.0 / (sig * sig));
    rc.two_inv_s2 = 2.f * rc.inv_s2;
    rc.lowpass_mode = s.lowpass_mode;
    rc.batch = s.batch_depth;
    rc.esm_c = s.esm_c;
    rc.esm_bias = s.esm_bias;
    rc.alpha_min_d = (double)s.alpha_min;
    rc.sigma_d = sig;
    rc.det_rel_eps_d = (double)s.det_rel_eps;
    return rc;
}

static ss_status check_call(ss_plan *p, const ss_surfels *s, const ss_views *v)
{
    if (!p) return fail(SS_ERR_INVALID_ARG, "plan is NULL");
    if (!p->ws) return fail(SS_ERR_STATE, "no workspace bound");
    if (!s || !v) return fail(SS_ERR_INVALID_ARG, "surfels or views is NULL");
    if (s->n != p->n) return fail(SS_ERR_INVALID_ARG, "surfel count differs from the plan");
    if (v->n != p->nv) return fail(SS_ERR_INVALID_ARG, "view count differs from the plan");
    if (p->n > 0 && (!s->mean || !s->t_u || !s->t_v || !s->scale || !s->opacity || !s->albedo))
        return fail(SS_ERR_INVALID_ARG, "a surfel array is NULL");
    if (!v->Fxy) return fail(SS_ERR_INVALID_ARG, "views.Fxy is NULL");
    if (!std::isfinite(v->b_z)) return fail(SS_ERR_INVALID_ARG, "b_z is not finite");
    if (v->width && v->height)
        for (int i = 0; i < p->nv; ++i)
            if (v->width[i] != p->W[i] || v->height[i] != p->H[i])
                return fail(SS_ERR_INVALID_ARG, "view sizes differ from the plan");
    if (hipSetDevice(p->ctx->device) != hipSuccess)
        return fail(SS_ERR_HIP, "hipSetDevice failed");
    return SS_OK;
}

// Centre-depth order and the gather of surfel parameters into depth-rank order.
static ss_status prepare(ss_plan *p, const ss_surfels *s, const ss_views *v, bool sun,
                         uint32_t **order_out, float **sorted_out, hipStream_t st)
{
    const Layout &L = p->L;
    uint32_t *ka = p->at<uint32_t>(sun ? L.sk_a : L.mk_a), *kb = p->at<uint32_t>(sun ? L.sk_b : L.mk_b);
    uint32_t *va = p->at<uint32_t>(sun ? L.sv_a : L.mv_a), *vb = p->at<uint32_t>(sun ? L.sv_b : L.mv_b);
    float *sorted = p->at<float>(sun ? L.sorted_sun : L.sorted_main);
    if (!sun && p->sun_order_shared) {   // a shadow binning that read these buffers goes stale
        p->sun_valid = false;
        p->sun_order_shared = false;
    }
    StageScope scope(p, SS_STAGE_DEPTH_SORT, st);
    SS_HIP(launch_depth_keys(s->mean, p->n, v->b_z, ka, va, st));
    bool in_b = false;
    SS_HIP(radix_sort_pairs(ka, va, kb, vb, p->n, nullptr, p->n, 32, p->at<void>(L.radix_temp),
                            &in_b, st));
    uint32_t *order = in_b ? vb : va;
    SurfelPtrs sp{s->mean, s->t_u, s->t_v, s->scale, s->opacity, s->albedo, p->n};
    SS_HIP(launch_gather_params(order, sp, sorted, st));
    *order_out = order;
    *sorted_out = sorted;
    return SS_OK;
}

// Projection + pair-count scan (+ emission, tile sort and ranges when `bin`).
static ss_status bin_views(ss_plan *p, const ss_views *v, bool sun, const uint32_t *order,
                           const float *sorted, const float *vis, bool bin, hipStream_t st,
                           const uint32_t *tmask = nullptr)
{
    const Layout &L = p->L;
    const RasterConsts rc = consts(p->st);
    const ViewDesc *views = p->at<ViewDesc>(sun ? L.views_sun : L.views_main);
    float *rec = p->at<float>(sun ? L.rec_sun : L.rec_main);
    short4 *tiles = p->at<short4>(sun ? L.tiles_sun : L.tiles_main);
    uint32_t *counts = p->at<uint32_t>(sun ? L.counts_sun : L.counts_main);
    uint32_t *offs = p->at<uint32_t>(sun ? L.offs_sun : L.offs_main);
    unsigned long long *counters = p->at<unsigned long long>(L.counters);
    uint32_t *flags = p->at<uint32_t>(L.flags);
    const int64_t cap = sun ? p->cap_sun : p->cap_main;
    {
        StageScope scope(p, sun ? SS_STAGE_SUN_PROJECT : SS_STAGE_PROJECT, st);
        const float *vis_rank = nullptr;
        if (!sun && vis) {
            SS_HIP(launch_vis_to_rank(vis, p->n, p->nv, order, p->at<uint32_t>(L.inv_order),
                                      p->at<float>(L.vis_rank), st));
            vis_rank = p->at<float>(L.vis_rank);
        }
        SS_HIP(launch_project(sorted, p->n, p->nv, views, v->Fxy, sun ? nullptr : v->dF,
                              sun ? p->at<SunCam>(L.suncam) : nullptr, vis_rank,
                              v->b_z, p->st.tile_size, rc, rec, tiles, counts, tmask, st));
    }
    StageScope scope(p, sun ? SS_STAGE_SUN_BIN : SS_STAGE_BIN, st);
    SS_HIP(scan_pair_counts(counts, p->n, p->nv, offs, p->at<uint32_t>(L.scanparts), counters,
                            sun ? 1 : 0, flags + (sun ? 1 : 0), bin ? (uint64_t)cap : ~0ull, st));
    if (!bin) return SS_OK;
    uint32_t *ka = p->at<uint32_t>(sun ? L.qk_a : L.pk_a), *va = p->at<uint32_t>(sun ? L.qv_a : L.pv_a);
    uint32_t *kb = p->at<uint32_t>(sun ? L.qk_b : L.pk_b), *vb = p->at<uint32_t>(sun ? L.qv_b : L.pv_b);
    // pairs arrive grouped by view (the count scan is view-major) and in depth-rank order
    // inside a view, so a stable sort on the tile id inside each view's run is the whole
    // bucketing; its last pass also writes each tile's list range.  Views of at most 2^16
    // tiles sort 16-bit keys local to the view (a quarter less traffic per pass).
    const int32_t ntiles = sun ? p->tiles_sun : p->tiles_main;
    int64_t view_tiles = 1;
    for (const ViewDesc &d : sun ? p->vsun : p->vmain)
        view_tiles = std::max<int64_t>(view_tiles, (int64_t)d.tiles_x * d.tiles_y);
    const bool keys16 = view_tiles <= 65536;
    SS_HIP(launch_emit(order, p->n, p->nv, views, tiles, counts, offs, (uint64_t)cap, ka, keys16, va,
                       tmask, st));
    SortSegments seg{offs, p->n, p->nv, views,
                     p->at<uint32_t>(sun ? L.ranges_sun : L.ranges_main), ntiles};
    bool in_b = false;
    if (keys16)
        SS_HIP(radix_sort_pairs(reinterpret_cast<uint16_t *>(ka), va, reinterpret_cast<uint16_t *>(kb), vb,
                                cap, counters + (sun ? 1 : 0), 0, bits_for(view_tiles),
                                p->at<void>(L.radix_temp), &in_b, st, &seg));
    else
        SS_HIP(radix_sort_pairs(ka, va, kb, vb, cap, counters + (sun ? 1 : 0), 0, bits_for(view_tiles),
                                p->at<void>(L.radix_temp), &in_b, st, &seg));
    uint32_t *lists = in_b ? vb : va;
    if (sun) p->lists_sun = lists; else p->lists_main = lists;
    const uint32_t *torder = nullptr;
    if (p->st.tile_order == 1) {
        uint32_t *o = p->at<uint32_t>(sun ? L.torder_sun : L.torder_main);
        SS_HIP(launch_tile_order(p->at<uint32_t>(sun ? L.ranges_sun : L.ranges_main), ntiles,
                                 counters + (sun ? 1 : 0), !sun, o, p->at<uint32_t>(L.torder_parts), st));
        torder = o;
    }
    if (sun) p->torder_sun = torder; else p->torder_main = torder;
    return SS_OK;
}

// Contributor masks exist for 8x8 tiles when the workspace was laid out for them at the
// current pair capacity (a tile-size change keeps the layout: then the box test is used).
static unsigned long long *cmask_ptr(const ss_plan *p)
{
    if (p->st.tile_size != 8 || p->L.cmask_bytes < cmask_words(p->cap_main, p->tiles_main_max) * 8)
        return nullptr;
    return p->at<unsigned long long>(p->L.cmask);
}

static ss_status upload_views(ss_plan *p)
{
    if (!p->ws) return SS_OK;
    SS_HIP(hipSetDevice(p->ctx->device));
    SS_HIP(hipMemcpy(p->at<void>(p->L.views_main), p->vmain.data(), p->nv * sizeof(ViewDesc),
                     hipMemcpyHostToDevice));
    SS_HIP(hipMemcpy(p->at<void>(p->L.views_sun), p->vsun.data(), p->nv * sizeof(ViewDesc),
                     hipMemcpyHostToDevice));
    SS_HIP(hipMemset(p->at<void>(p->L.counters), 0, 16 * sizeof(unsigned long long)));
    SS_HIP(hipMemset(p->at<void>(p->L.flags), 0, 16 * sizeof(uint32_t)));
    return SS_OK;
}

// ------------------------------------------------------------------ surrogate MLP
// Byte offsets of the MLP's buffers for batches of up to `maxp` points: BF16 / FP32 weight
// copies, saved features and activations, logits, activation gradients, per-block partial
// weight gradients and output-layer partials.  constexpr so that the allocation-free
// training entry point can size its static scratch array at compile time.
struct MlpLayout {
    size_t o_wb = 0, o_wf = 0, o_F = 0, o_H = 0, o_logit = 0, o_dA = 0, o_pdw = 0, o_pdb = 0,
           o_pout = 0, total = 0;
};

static constexpr MlpLayout mlp_layout_for(int64_t maxp)
{
    MlpLayout L{};
    size_t o = 0;
    auto take = [&o](size_t b) { size_t r = o; o += (b + 255) & ~size_t(255); return r; };
    const size_t M = (size_t)(maxp > 0 ? maxp : 0);
    const size_t nblk = (M + kDwChunk - 1) / kDwChunk;   // mlp_dw_blocks(M)
    const size_t nout = (M + 255) / 256;
    L.o_wb = take(kMlpBf16 * 2);
    L.o_wf = take(kMlpF32 * 4);
    L.o_F = take(M * kMlpIn * 2);
    L.o_H = take(3 * M * kMlpWidth * 2);
    L.o_logit = take(M * 4);
    L.o_dA = take(2 * M * kMlpWidth * 2);
    L.o_pdw = take(nblk * kMlpWidth * kMlpIn * 4);
    L.o_pdb = take(nblk * kMlpWidth * 4);
    L.o_pout = take(nout * 66 * 4);
    L.total = o;
    return L;
}

// Allocation-free MLP backward (ss_mlp_backward_noalloc): its buffers live in this fixed
// device array, laid out for batches of up to kNoAllocMaxPoints points (15.1 MiB), not in
// a bound workspace.  Every device holds its own copy.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): the device
// address comes from hipGetSymbolAddress, once per device, when a context is created on
// it (scratch_address), and only that address is used.
constexpr int64_t kNoAllocMaxPoints = 16384;
constexpr MlpLayout kNoAllocLayout = mlp_layout_for(kNoAllocMaxPoints);
static __device__ __align__(256) char scratch[kNoAllocLayout.total];
static_assert(kNoAllocLayout.total <= (size_t(16) << 20), "no-alloc scratch must stay modest");

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device`, looked up once with that device current.
static ss_status scratch_address(int device, char **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return SS_OK;   // entry point refuses later
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        SS_HIP(hipSetDevice(device));
        SS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(SS_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[device] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return SS_OK;
}

struct ss_mlp {
    ss_context *ctx = nullptr;
    ss_mlp_config cfg{};
    char *ws = nullptr;
    size_t bytes = 0;
    int64_t maxp = 0;
    MlpLayout L{};
    template <class T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

static void mlp_layout(ss_mlp *m, int64_t maxp) { m->L = mlp_layout_for(maxp); }

static MlpNorm mlp_norm(const ss_mlp *m)
{
    return MlpNorm{m->cfg.centre[0], m->cfg.centre[1], m->cfg.centre[2], m->cfg.inv_half};
}

// ======================================================================= C ABI
extern "C" {

const char *ss_last_error(void) { return g_err.c_str(); }

void ss_default_settings(ss_raster_settings *out)
{
    if (!out) return;
    std::memset(out, 0, sizeof *out);
    out->struct_size = sizeof(ss_raster_settings);
    out->tile_size = 16;
    out->batch_depth = 64;
    out->alpha_min = 1.0f / 255.0f;
    out->alpha_max = 0.99f;
    out->T_min = 1e-4f;
    out->lowpass_sigma = 0.70710678f;
    out->lowpass_mode = 0;
    out->det_rel_eps = 1e-6f;
    out->esm_c = 2.0f;
    out->esm_bias = 0.5f;
    out->sun_map_size = 1024;
    out->tile_order = 0;
}

ss_status ss_context_create(int32_t device, ss_context **out)
{
    if (!out) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(SS_ERR_HIP, "no HIP device");
    if (device < 0 || device >= count) return fail(SS_ERR_INVALID_ARG, "device out of range");
    hipDeviceProp_t prop;
    SS_HIP(hipGetDeviceProperties(&prop, device));
    std::string arch = prop.gcnArchName;
    if (arch.rfind("gfx950", 0) != 0)
        return fail(SS_ERR_UNSUPPORTED, "device is " + arch + ", this library is built for gfx950");
    char *scr = nullptr;
    ss_status e = scratch_address(device, &scr);
    if (e != SS_OK) return e;
    auto *c = new ss_context;
    c->device = device;
    c->cus = prop.multiProcessorCount;
    c->arch = arch;
    c->scratch = scr;
    *out = c;
    return SS_OK;
}

ss_status ss_context_destroy(ss_context *ctx)
{
    delete ctx;
    return SS_OK;
}

ss_status ss_plan_create(ss_context *ctx, int64_t n_surfels, int32_t n_views,
                         const int32_t *width, const int32_t *height,
                         const ss_raster_settings *settings, ss_plan **out)
{
    if (!out) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(SS_ERR_INVALID_ARG, "context is NULL");
    if (n_surfels < 0 || n_surfels > 0x7FFFFFFF)
        return fail(SS_ERR_INVALID_ARG, "n_surfels must be in [0, 2^31)");
    if (n_views < 1 || n_views > 65535) return fail(SS_ERR_INVALID_ARG, "n_views must be in [1, 65535]");
    if (!width || !height) return fail(SS_ERR_INVALID_ARG, "width/height is NULL");
    ss_status e = check_settings(settings);
    if (e != SS_OK) return e;
    int64_t tiles = 0;
    for (int v = 0; v < n_views; ++v) {
        if (width[v] < 1 || width[v] > 32767 || height[v] < 1 || height[v] > 32767)
            return fail(SS_ERR_INVALID_ARG, "view sides must be in [1, 32767]");
        tiles += (int64_t)((width[v] + 7) / 8) * ((height[v] + 7) / 8);
    }
    const int64_t S = settings->sun_map_size;
    if (tiles > 0x7FFFFFFF || (int64_t)n_views * ((S + 7) / 8) * ((S + 7) / 8) > 0x7FFFFFFF)
        return fail(SS_ERR_INVALID_ARG, "too many tiles");
    auto *p = new ss_plan;
    p->ctx = ctx;
    p->st = *settings;
    p->n = n_surfels;
    p->nv = n_views;
    p->W.assign(width, width + n_views);
    p->H.assign(height, height + n_views);
    build_views(p);
    max_tiles(p);
    *out = p;
    return SS_OK;
}

ss_status ss_plan_destroy(ss_plan *plan)
{
    delete plan;
    return SS_OK;
}

ss_status ss_plan_set_settings(ss_plan *p, const ss_raster_settings *settings)
{
    if (!p) return fail(SS_ERR_INVALID_ARG, "plan is NULL");
    ss_status e = check_settings(settings);
    if (e != SS_OK) return e;
    if (settings->sun_map_size != p->st.sun_map_size)
        return fail(SS_ERR_INVALID_ARG, "sun_map_size is fixed at plan creation");
    p->st = *settings;
    build_views(p);
    p->fwd_valid = p->sun_valid = false;
    ++p->generation;
    return upload_views(p);
}

ss_status ss_plan_workspace_size(ss_plan *p, int64_t main_pairs, int64_t sun_pairs, size_t *bytes)
{
    if (!p || !bytes) return fail(SS_ERR_INVALID_ARG, "plan or bytes is NULL");
    if (main_pairs < 0 || sun_pairs < 0 || main_pairs > 0xFFFFFFFFll || sun_pairs > 0xFFFFFFFFll)
        return fail(SS_ERR_INVALID_ARG, "pair capacity must be in [0, 2^32)");
    *bytes = make_layout(p, main_pairs, sun_pairs).total;
    return SS_OK;
}

ss_status ss_plan_bind_workspace(ss_plan *p, void *workspace, size_t bytes, int64_t main_pairs,
                                 int64_t sun_pairs)
{
    if (!p || !workspace) return fail(SS_ERR_INVALID_ARG, "plan or workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(SS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (main_pairs < 0 || sun_pairs < 0 || main_pairs > 0xFFFFFFFFll || sun_pairs > 0xFFFFFFFFll)
        return fail(SS_ERR_INVALID_ARG, "pair capacity must be in [0, 2^32)");
    Layout L = make_layout(p, main_pairs, sun_pairs);
    if (bytes < L.total) return fail(SS_ERR_CAPACITY, "workspace smaller than required");
    p->L = L;
    p->ws = reinterpret_cast<char *>(workspace);
    p->ws_bytes = bytes;
    p->cap_main = main_pairs;
    p->cap_sun = sun_pairs;
    p->fwd_valid = p->sun_valid = false;
    ++p->generation;
    return upload_views(p);
}

ss_status ss_count_pairs(ss_plan *p, const ss_surfels *s, const ss_views *v, int64_t *main_pairs,
                         int64_t *sun_pairs, ss_stream stream)
{
    ss_status e = check_call(p, s, v);
    if (e != SS_OK) return e;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint32_t *order;
    float *sorted;
    e = prepare(p, s, v, false, &order, &sorted, st);
    if (e != SS_OK) return e;
    e = bin_views(p, v, false, order, sorted, nullptr, false, st);
    if (e != SS_OK) return e;
    if (v->sun) {
        e = prepare(p, s, v, true, &order, &sorted, st);
        if (e != SS_OK) return e;
        SS_HIP(launch_sun_cameras(s->mean, p->n, p->nv, v->Fxy, v->dF, v->sun, v->b_z,
                                  p->st.sun_map_size, p->at<double>(p->L.bounds),
                                  p->at<SunCam>(p->L.suncam), st));
        e = bin_views(p, v, true, order, sorted, nullptr, false, st);
        if (e != SS_OK) return e;
    }
    unsigned long long c[2] = {0, 0};
    SS_HIP(hipMemcpyAsync(c, p->at<void>(p->L.counters), sizeof c, hipMemcpyDeviceToHost, st));
    SS_HIP(hipStreamSynchronize(st));
    if (main_pairs) *main_pairs = (int64_t)c[0];
    if (sun_pairs) *sun_pairs = v->sun ? (int64_t)c[1] : 0;
    p->fwd_valid = p->sun_valid = false;
    return SS_OK;
}

ss_status ss_plan_check(ss_plan *p, int32_t *overflowed, int64_t *main_pairs, int64_t *sun_pairs,
                        ss_stream stream)
{
    if (!p || !p->ws) return fail(SS_ERR_STATE, "plan has no workspace");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    SS_HIP(hipSetDevice(p->ctx->device));
    unsigned long long c[2];
    uint32_t f[2];
    SS_HIP(hipMemcpyAsync(c, p->at<void>(p->L.counters), sizeof c, hipMemcpyDeviceToHost, st));
    SS_HIP(hipMemcpyAsync(f, p->at<void>(p->L.flags), sizeof f, hipMemcpyDeviceToHost, st));
    SS_HIP(hipStreamSynchronize(st));
    if (overflowed) *overflowed = (f[0] | f[1]) ? 1 : 0;
    if (main_pairs) *main_pairs = (int64_t)c[0];
    if (sun_pairs) *sun_pairs = (int64_t)c[1];
    return SS_OK;
}

}  // extern "C"

// Forward of all views; with `order` given (ss_step) the depth order and rank-ordered
// parameters already in the main-view buffers are used, else they are computed here.
static ss_status forward_pass(ss_plan *p, const ss_surfels *s, const ss_views *v, const float *vis,
                              float *image, float *albedo_out, float *vis_out, float *depth,
                              float *normal, float *T_final, int32_t *last, hipStream_t st,
                              uint32_t *order, float *sorted, const DistArgs *dist = nullptr)
{
    ss_status e;
    p->fwd_valid = false;
    SS_HIP(fill_u32(p->at<uint32_t>(p->L.flags), 0u, 1, st));
    unsigned long long *stat = p->at<unsigned long long>(p->L.stat_main);
    SS_HIP(fill_u32(reinterpret_cast<uint32_t *>(stat), 0u, 2 * kStatSlots * kStatStride, st));
    if (!order && (e = prepare(p, s, v, false, &order, &sorted, st)) != SS_OK) return e;
    if ((e = bin_views(p, v, false, order, sorted, vis, true, st)) != SS_OK) return e;
    RasterConsts rc = consts(p->st);
    rc.torder = p->torder_main;
    {
        StageScope scope(p, SS_STAGE_RASTER_FWD, st);
        SS_HIP(launch_raster_fwd(p->st.tile_size, false, vis != nullptr, p->tiles_main, p->nv,
                                 p->at<ViewDesc>(p->L.views_main),
                                 p->at<uint32_t>(p->L.ranges_main), p->lists_main,
                                 p->at<float>(p->L.rec_main), p->n, rc, v->colC, v->colc,
                                 v->ambient, nullptr, image, albedo_out, vis_out, depth, normal,
                                 T_final, last, stat, cmask_ptr(p), st, dist));
    }
    p->order_main = order;
    p->fwd_valid = true;
    return SS_OK;
}

extern "C" {

ss_status ss_forward(ss_plan *p, const ss_surfels *s, const ss_views *v, const float *vis,
                     float *image, float *albedo_out, float *vis_out, float *depth,
                     float *normal, float *T_final, int32_t *last, ss_stream stream)
{
    ss_status e = check_call(p, s, v);
    if (e != SS_OK) return e;
    if (!image || !albedo_out || !vis_out || !depth || !normal || !T_final || !last)
        return fail(SS_ERR_INVALID_ARG, "an output pointer is NULL");
    return forward_pass(p, s, v, vis, image, albedo_out, vis_out, depth, normal, T_final, last,
                        reinterpret_cast<hipStream_t>(stream), nullptr, nullptr);
}

static ss_status geom_args(const ss_plan *p, const ss_geom_io *geom, bool fwd, DistArgs *out)
{
    if (!geom || geom->struct_size != sizeof(ss_geom_io))
        return fail(SS_ERR_INVALID_ARG, "bad ss_geom_io");
    if (!(geom->depth_scale > 0.f) || !std::isfinite(geom->depth_scale))
        return fail(SS_ERR_INVALID_ARG, "depth_scale must be positive");
    if (!geom->aux || (fwd && !geom->dist))
        return fail(SS_ERR_INVALID_ARG, "geom->aux (and, in the forward, geom->dist) is required");
    *out = DistArgs{geom->depth_scale, geom->dist, geom->aux, geom->d_dist, p->P};
    return SS_OK;
}

ss_status ss_forward_geom(ss_plan *p, const ss_surfels *s, const ss_views *v, const float *vis,
                          float *image, float *albedo_out, float *vis_out, float *depth,
                          float *normal, float *T_final, int32_t *last, const ss_geom_io *geom,
                          ss_stream stream)
{
    ss_status e = check_call(p, s, v);
    if (e != SS_OK) return e;
    if (!image || !albedo_out || !vis_out || !depth || !normal || !T_final || !last)
        return fail(SS_ERR_INVALID_ARG, "an output pointer is NULL");
    DistArgs da;
    if ((e = geom_args(p, geom, true, &da)) != SS_OK) return e;
    return forward_pass(p, s, v, vis, image, albedo_out, vis_out, depth, normal, T_final, last,
                        reinterpret_cast<hipStream_t>(stream), nullptr, nullptr, &da);
}

static ss_status backward_pass(ss_plan *p, const ss_surfels *s, const ss_views *v, const float *vis,
                               const float *albedo_out, const float *vis_out, const float *T_final,
                               const int32_t *last, const float *d_image, const float *d_depth,
                               const float *d_normal, float *d_mean, float *d_t_u, float *d_t_v,
                               float *d_scale, float *d_opacity, float *d_albedo, float *d_dF,
                               float *d_colC, float *d_colc, float *d_ambient, ss_stream stream,
                               const DistArgs *dist)
{
    ss_status e = check_call(p, s, v);
    if (e != SS_OK) return e;
    if (!p->fwd_valid) return fail(SS_ERR_STATE, "backward needs the plan's forward binning");
    if (!albedo_out || !vis_out || !T_final || !last)
        return fail(SS_ERR_INVALID_ARG, "a saved forward output is NULL");
    if ((p->n > 0 && (!d_mean || !d_t_u || !d_t_v || !d_scale || !d_opacity || !d_albedo)) ||
        !d_dF || !d_colC || !d_colc || !d_ambient)
        return fail(SS_ERR_INVALID_ARG, "a gradient output is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const Layout &L = p->L;
    RasterConsts rc = consts(p->st);
    rc.torder = p->torder_main;
    float *recgrad = p->at<float>(L.recgrad);
    {
        StageScope scope(p, SS_STAGE_REDUCE, st);
        SS_HIP(fill_f32(recgrad, 0.f, p->n * (int64_t)p->nv * kGradFloats, st));
    }
    {
        StageScope scope(p, SS_STAGE_RASTER_BWD, st);
        SS_HIP(launch_raster_bwd(p->st.tile_size, vis != nullptr, p->tiles_main, p->nv,
                                 p->at<ViewDesc>(L.views_main), p->at<uint32_t>(L.ranges_main),
                                 p->lists_main, p->at<float>(L.rec_main), p->n, rc, v->colC,
                                 v->colc, v->ambient, albedo_out, vis_out, T_final, last, d_image,
                                 d_depth, d_normal, recgrad, p->at<float>(L.colour_parts),
                                 cmask_ptr(p), st, dist));
    }
    {
        StageScope scope(p, SS_STAGE_REDUCE, st);
        SS_HIP(launch_colour_reduce(p->at<float>(L.colour_parts), p->nv,
                                    p->at<ViewDesc>(L.views_main), d_colC, d_colc, d_ambient, st));
    }
    {
        StageScope scope(p, SS_STAGE_PROJECT_BWD, st);
        SS_HIP(launch_project_bwd(p->at<float>(L.sorted_main), p->n, p->order_main, p->nv, v->Fxy,
                                  v->dF, consts(p->st).det_rel_eps_d, recgrad, d_mean, d_t_u, d_t_v,
                                  d_scale, d_opacity, d_albedo, p->at<float>(L.dF_parts), st));
    }
    StageScope scope(p, SS_STAGE_REDUCE, st);
    SS_HIP(launch_dF_reduce(p->at<float>(L.dF_parts), project_bwd_blocks(p->n), p->nv, d_dF, st));
    return SS_OK;
}

ss_status ss_backward(ss_plan *p, const ss_surfels *s, const ss_views *v, const float *vis,
                      const float *albedo_out, const float *vis_out, const float *T_final,
                      const int32_t *last, const float *d_image, const float *d_depth,
                      const float *d_normal, float *d_mean, float *d_t_u, float *d_t_v,
                      float *d_scale, float *d_opacity, float *d_albedo, float *d_dF,
                      float *d_colC, float *d_colc, float *d_ambient, ss_stream stream)
{
    return backward_pass(p, s, v, vis, albedo_out, vis_out, T_final, last, d_image, d_depth,
                         d_normal, d_mean, d_t_u, d_t_v, d_scale, d_opacity, d_albedo, d_dF,
                         d_colC, d_colc, d_ambient, stream, nullptr);
}

ss_status ss_backward_geom(ss_plan *p, const ss_surfels *s, const ss_views *v, const float *vis,
                           const float *albedo_out, const float *vis_out, const float *T_final,
                           const int32_t *last, const float *d_image, const float *d_depth,
                           const float *d_normal, const ss_geom_io *geom, float *d_mean,
                           float *d_t_u, float *d_t_v, float *d_scale, float *d_opacity,
                           float *d_albedo, float *d_dF, float *d_colC, float *d_colc,
                           float *d_ambient, ss_stream stream)
{
    if (!p) return fail(SS_ERR_INVALID_ARG, "plan is NULL");
    DistArgs da;
    ss_status e = geom_args(p, geom, false, &da);
    if (e != SS_OK) return e;
    return backward_pass(p, s, v, vis, albedo_out, vis_out, T_final, last, d_image, d_depth,
                         d_normal, d_mean, d_t_u, d_t_v, d_scale, d_opacity, d_albedo, d_dF,
                         d_colC, d_colc, d_ambient, stream, &da);
}

ss_status ss_normal_loss(ss_plan *p, const ss_views *v, const float *depth, const float *T_final,
                         const float *normal, float weight, float tau, float *loss,
                         float *normal_d, float *d_depth, float *d_normal, float *d_dF,
                         ss_stream stream)
{
    if (!p) return fail(SS_ERR_INVALID_ARG, "plan is NULL");
    if (!p->ws) return fail(SS_ERR_STATE, "no workspace bound");
    if (!v || v->n != p->nv || !v->Fxy) return fail(SS_ERR_INVALID_ARG, "views invalid");
    if (!depth || !T_final || !normal || !loss || !d_depth || !d_normal)
        return fail(SS_ERR_INVALID_ARG, "a map, the loss or a gradient pointer is NULL");
    if (!std::isfinite(weight) || !(tau > 0.f && tau <= 1.f))
        return fail(SS_ERR_INVALID_ARG, "weight must be finite and tau in (0, 1]");
    SS_HIP(hipSetDevice(p->ctx->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const Layout &L = p->L;
    StageScope scope(p, SS_STAGE_NORMAL_LOSS, st);
    SS_HIP(launch_normal_loss(p->at<ViewDesc>(L.views_main), p->vmain.data(), p->nv, max_view_pixels(p), v->Fxy,
                              v->dF, depth, T_final, normal, weight, tau,
                              p->at<GeomCam>(L.geom_cams), p->at<float2>(L.geom_seeds),
                              p->at<double>(L.geom_parts), loss, normal_d, d_depth, d_normal,
                              d_dF, st));
    return SS_OK;
}

}  // extern "C"

// Plain shadow pass; with `order` given (ss_step: the main-view depth order of the same
// surfels, the order is view independent) no depth sort runs here.
static ss_status shadow_pass(ss_plan *p, const ss_surfels *s, const ss_views *v, float *sun_depth,
                             float *vis, hipStream_t st, uint32_t *order, float *sorted)
{
    ss_status e;
    const Layout &L = p->L;
    p->sun_valid = false;
    SS_HIP(fill_u32(p->at<uint32_t>(L.flags) + 1, 0u, 1, st));
    unsigned long long *stat = p->at<unsigned long long>(L.stat_sun);
    SS_HIP(fill_u32(reinterpret_cast<uint32_t *>(stat), 0u, 2 * kStatSlots * kStatStride, st));
    const bool shared = order != nullptr;
    if (!shared && (e = prepare(p, s, v, true, &order, &sorted, st)) != SS_OK) return e;
    {
        StageScope scope(p, SS_STAGE_SUN_CAMERA, st);
        SS_HIP(launch_sun_cameras(s->mean, p->n, p->nv, v->Fxy, v->dF, v->sun, v->b_z,
                                  p->st.sun_map_size, p->at<double>(L.bounds),
                                  p->at<SunCam>(L.suncam), st));
    }
    if ((e = bin_views(p, v, true, order, sorted, nullptr, true, st)) != SS_OK) return e;
    float *D = sun_depth ? sun_depth : p->at<float>(L.sun_depth);
    RasterConsts rc = consts(p->st);
    rc.torder = p->torder_sun;
    {
        StageScope scope(p, SS_STAGE_SUN_RASTER, st);
        SS_HIP(launch_raster_fwd(p->st.tile_size, true, false, p->tiles_sun, p->nv,
                                 p->at<ViewDesc>(L.views_sun), p->at<uint32_t>(L.ranges_sun),
                                 p->lists_sun, p->at<float>(L.rec_sun), p->n, rc, nullptr, nullptr,
                                 nullptr, p->at<SunCam>(L.suncam), nullptr, nullptr, nullptr, D,
                                 nullptr, nullptr, nullptr, stat, nullptr, st));
    }
    {
        StageScope scope(p, SS_STAGE_SHADOW_QUERY, st);
        SS_HIP(launch_shadow_query(s->mean, p->n, p->nv, p->at<SunCam>(L.suncam), D,
                                   p->st.sun_map_size, v->b_z, p->st.esm_c, p->st.esm_bias, vis,
                                   0.f, st));
    }
    p->order_sun = order;
    p->sun_order_shared = shared;
    p->sun_valid = true;
    return SS_OK;
}

extern "C" {

ss_status ss_shadow_plain(ss_plan *p, const ss_surfels *s, const ss_views *v, float *sun_depth,
                          float *vis, ss_stream stream)
{
    ss_status e = check_call(p, s, v);
    if (e != SS_OK) return e;
    if (!v->sun) return fail(SS_ERR_INVALID_ARG, "views.sun is NULL");
    if (!vis) return fail(SS_ERR_INVALID_ARG, "vis output is NULL");
    return shadow_pass(p, s, v, sun_depth, vis, reinterpret_cast<hipStream_t>(stream), nullptr,
                       nullptr);
}

ss_status ss_debug_binning(ss_plan *p, int32_t which, uint32_t *order, int32_t *surf_tiles,
                           uint32_t *tile_ranges, uint32_t *tile_lists, float *records,
                           int64_t *n_tiles, int64_t *n_pairs, ss_stream stream)
{
    if (!p || !p->ws) return fail(SS_ERR_STATE, "plan has no workspace");
    if (which != 0 && which != 1) return fail(SS_ERR_INVALID_ARG, "which must be 0 or 1");
    const bool sun = which == 1;
    if (!(sun ? p->sun_valid : p->fwd_valid)) return fail(SS_ERR_STATE, "no binning to report");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    SS_HIP(hipSetDevice(p->ctx->device));
    const Layout &L = p->L;
    const uint32_t *ord = sun ? p->order_sun : p->order_main;
    const int64_t nt = sun ? p->tiles_sun : p->tiles_main;
    const int64_t cap = sun ? p->cap_sun : p->cap_main;
    const unsigned long long *cnt = p->at<unsigned long long>(L.counters) + (sun ? 1 : 0);
    unsigned long long k = 0;
    SS_HIP(hipMemcpyAsync(&k, cnt, sizeof k, hipMemcpyDeviceToHost, st));
    SS_HIP(hipStreamSynchronize(st));
    const int64_t npairs = (int64_t)std::min<unsigned long long>(k, (unsigned long long)cap);
    if (n_tiles) *n_tiles = nt;
    if (n_pairs) *n_pairs = npairs;
    if (order && p->n > 0)
        SS_HIP(hipMemcpyAsync(order, ord, p->n * 4, hipMemcpyDeviceToDevice, st));
    if (surf_tiles && p->n > 0)
        SS_HIP(launch_unpermute_tiles(ord, p->n, p->nv, p->at<short4>(sun ? L.tiles_sun : L.tiles_main),
                                      surf_tiles, st));
    if (tile_ranges)
        SS_HIP(hipMemcpyAsync(tile_ranges, p->at<void>(sun ? L.ranges_sun : L.ranges_main), nt * 8,
                              hipMemcpyDeviceToDevice, st));
    if (tile_lists && npairs > 0)
        SS_HIP(launch_map_through(ord, p->n, cnt, cap, sun ? p->lists_sun : p->lists_main, tile_lists,
                                  st));
    if (records && p->n > 0)
        SS_HIP(launch_unpermute_rows(ord, p->n, p->nv, p->at<uint32_t>(sun ? L.rec_sun : L.rec_main),
                                     4 * (sun ? kSunRecStride4 : kRecStride4), kRecFloats,
                                     reinterpret_cast<uint32_t *>(records), st));
    SS_HIP(hipStreamSynchronize(st));
    return SS_OK;
}

ss_status ss_debug_sun_cameras(ss_plan *p, double *out, ss_stream stream)
{
    if (!p || !p->ws || !out) return fail(SS_ERR_INVALID_ARG, "plan/workspace/out missing");
    if (!p->sun_valid) return fail(SS_ERR_STATE, "no shadow pass has run");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    std::vector<SunCam> c(p->nv);
    SS_HIP(hipMemcpyAsync(c.data(), p->at<void>(p->L.suncam), p->nv * sizeof(SunCam),
                          hipMemcpyDeviceToHost, st));
    SS_HIP(hipStreamSynchronize(st));
    for (int v = 0; v < p->nv; ++v) {
        for (int k = 0; k < 6; ++k) out[9 * v + k] = c[v].B[k];
        out[9 * v + 6] = c[v].b[0];
        out[9 * v + 7] = c[v].b[1];
        out[9 * v + 8] = c[v].zfar;
    }
    return SS_OK;
}

// ----------------------------------------------------------- step / graph / tune
struct ss_graph {
    ss_plan *plan = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t generation = 0;   // the plan's generation at capture
};

static ss_status check_io(const ss_plan *p, const ss_views *v, const ss_step_io *io)
{
    if (!io || io->struct_size != sizeof(ss_step_io)) return fail(SS_ERR_INVALID_ARG, "bad ss_step_io");
    if (v && v->sun && !io->vis) return fail(SS_ERR_INVALID_ARG, "io->vis is required with views->sun");
    (void)p;
    return SS_OK;
}

ss_status ss_step(ss_plan *p, const ss_surfels *s, const ss_views *v, const ss_step_io *io,
                  ss_stream stream)
{
    ss_status e = check_io(p, v, io);
    if (e != SS_OK) return e;
    if ((e = check_call(p, s, v)) != SS_OK) return e;
    if (!io->image || !io->albedo_out || !io->vis_out || !io->depth || !io->normal ||
        !io->T_final || !io->last)
        return fail(SS_ERR_INVALID_ARG, "an output pointer is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // one depth order per step, shared by the sun maps and the views (Sec. 3.3: the
    // depth row is fixed, so the centre-depth order does not depend on the view)
    uint32_t *order;
    float *sorted;
    if ((e = prepare(p, s, v, false, &order, &sorted, st)) != SS_OK) return e;
    if (v->sun && (e = shadow_pass(p, s, v, io->sun_depth, io->vis, st, order, sorted)) != SS_OK)
        return e;
    e = forward_pass(p, s, v, io->vis, io->image, io->albedo_out, io->vis_out, io->depth,
                     io->normal, io->T_final, io->last, st, order, sorted);
    if (e != SS_OK) return e;
    return ss_backward(p, s, v, io->vis, io->albedo_out, io->vis_out, io->T_final, io->last,
                       io->d_image, io->d_depth, io->d_normal, io->d_mean, io->d_t_u, io->d_t_v,
                       io->d_scale, io->d_opacity, io->d_albedo, io->d_dF, io->d_colC, io->d_colc,
                       io->d_ambient, stream);
}

ss_status ss_graph_build(ss_plan *p, const ss_surfels *s, const ss_views *v, const ss_step_io *io,
                         ss_graph **out)
{
    if (!out) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    ss_status e = check_call(p, s, v);
    if (e != SS_OK) return e;
    if ((e = check_io(p, v, io)) != SS_OK) return e;
    hipStream_t cs = nullptr;
    SS_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const bool timing = p->timer.on;
    p->timer.on = false;
    hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) {
        p->timer.on = timing;
        (void)hipStreamDestroy(cs);
        return fail(SS_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(he));
    }
    e = ss_step(p, s, v, io, reinterpret_cast<ss_stream>(cs));
    hipGraph_t g = nullptr;
    he = hipStreamEndCapture(cs, &g);
    p->timer.on = timing;
    (void)hipStreamDestroy(cs);
    if (e != SS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    if (he != hipSuccess || !g)
        return fail(SS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he));
    hipGraphExec_t x = nullptr;
    he = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (he != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(SS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(he));
    }
    auto *G = new ss_graph;
    G->plan = p;
    G->graph = g;
    G->exec = x;
    G->generation = p->generation;
    *out = G;
    return SS_OK;
}

ss_status ss_graph_launch(ss_graph *G, ss_stream stream)
{
    if (!G || !G->exec) return fail(SS_ERR_INVALID_ARG, "graph is NULL");
    if (G->generation != G->plan->generation)
        return fail(SS_ERR_STATE, "the plan's workspace or settings changed since the graph "
                                  "was captured; rebuild the graph");
    SS_HIP(hipSetDevice(G->plan->ctx->device));
    SS_HIP(hipGraphLaunch(G->exec, reinterpret_cast<hipStream_t>(stream)));
    return SS_OK;
}

ss_status ss_graph_destroy(ss_graph *G)
{
    if (!G) return SS_OK;
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return SS_OK;
}

ss_status ss_autotune(ss_plan *p, const ss_surfels *s, const ss_views *v, const ss_step_io *io,
                      int32_t reps, ss_raster_settings *best, double *best_ms, double *table,
                      ss_stream stream)
{
    ss_status e = check_call(p, s, v);
    if (e != SS_OK) return e;
    if ((e = check_io(p, v, io)) != SS_OK) return e;
    if (reps < 1) reps = 1;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const ss_raster_settings base = p->st;
    const int tiles[3] = {8, 16, 32};
    const int batches[4] = {32, 64, 128, 256};
    hipEvent_t a = nullptr, b = nullptr;
    SS_HIP(hipEventCreate(&a));
    SS_HIP(hipEventCreate(&b));
    double best_t = -1.0;
    ss_raster_settings best_s = base;
    int row = 0;
    for (int ti = 0; ti < 3; ++ti) {
        for (int bi = 0; bi < 4; ++bi, ++row) {
            ss_raster_settings c = base;
            c.tile_size = tiles[ti];
            c.batch_depth = batches[bi];
            double ms = -1.0;
            if (c.batch_depth > c.tile_size * c.tile_size) {   // one staged record per thread
                if (table) {
                    table[3 * row] = c.tile_size;
                    table[3 * row + 1] = c.batch_depth;
                    table[3 * row + 2] = ms;
                }
                continue;
            }
            if ((e = ss_plan_set_settings(p, &c)) != SS_OK) break;
            int64_t km = 0, ks = 0;
            if ((e = ss_count_pairs(p, s, v, &km, &ks, stream)) != SS_OK) break;
            if (km <= p->cap_main && ks <= p->cap_sun) {
                if ((e = ss_step(p, s, v, io, stream)) != SS_OK) break;
                std::vector<double> t;
                for (int r = 0; r < reps; ++r) {
                    SS_HIP(hipEventRecord(a, st));
                    if ((e = ss_step(p, s, v, io, stream)) != SS_OK) break;
                    SS_HIP(hipEventRecord(b, st));
                    SS_HIP(hipEventSynchronize(b));
                    float f = 0.f;
                    SS_HIP(hipEventElapsedTime(&f, a, b));
                    t.push_back(f);
                }
                if (e != SS_OK) break;
                std::sort(t.begin(), t.end());
                ms = t[t.size() / 2];
                if (best_t < 0 || ms < best_t) { best_t = ms; best_s = c; }
            }
            if (table) {
                table[3 * row] = c.tile_size;
                table[3 * row + 1] = c.batch_depth;
                table[3 * row + 2] = ms;
            }
        }
        if (e != SS_OK) break;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != SS_OK) {
        (void)ss_plan_set_settings(p, &base);
        return e;
    }
    if (best_t < 0) {
        (void)ss_plan_set_settings(p, &base);
        return fail(SS_ERR_CAPACITY, "no candidate fits the bound pair capacities");
    }
    if ((e = ss_plan_set_settings(p, &best_s)) != SS_OK) return e;
    if (best) *best = best_s;
    if (best_ms) *best_ms = best_t;
    return SS_OK;
}

ss_status ss_mlp_create(ss_context *ctx, const ss_mlp_config *cfg, ss_mlp **out)
{
    if (!out) return fail(SS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx || !cfg || cfg->struct_size != sizeof(ss_mlp_config))
        return fail(SS_ERR_INVALID_ARG, "context or config invalid");
    if (!(cfg->inv_half > 0.f) || !std::isfinite(cfg->inv_half))
        return fail(SS_ERR_INVALID_ARG, "inv_half must be positive");
    auto *m = new ss_mlp;
    m->ctx = ctx;
    m->cfg = *cfg;
    *out = m;
    return SS_OK;
}

ss_status ss_mlp_destroy(ss_mlp *m)
{
    delete m;
    return SS_OK;
}

ss_status ss_mlp_workspace_size(ss_mlp *m, int64_t max_points, size_t *bytes)
{
    if (!m || !bytes || max_points < 0) return fail(SS_ERR_INVALID_ARG, "bad arguments");
    ss_mlp tmp;
    mlp_layout(&tmp, max_points);
    *bytes = tmp.L.total;
    return SS_OK;
}

ss_status ss_mlp_bind_workspace(ss_mlp *m, void *ws, size_t bytes, int64_t max_points)
{
    if (!m || !ws || max_points < 0) return fail(SS_ERR_INVALID_ARG, "bad arguments");
    if (((uintptr_t)ws & 255) != 0) return fail(SS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    mlp_layout(m, max_points);
    if (bytes < m->L.total) return fail(SS_ERR_CAPACITY, "workspace smaller than required");
    m->ws = reinterpret_cast<char *>(ws);
    m->bytes = bytes;
    m->maxp = max_points;
    return SS_OK;
}

ss_status ss_mlp_forward(ss_mlp *m, const float *w, const float *pts, int64_t n_pts,
                         const float *sun, int64_t n_sun, int32_t all_pairs, int32_t prob,
                         float *out, ss_stream stream)
{
    if (!m || !m->ws) return fail(SS_ERR_STATE, "MLP has no workspace");
    if (!w || !pts || !sun || !out) return fail(SS_ERR_INVALID_ARG, "NULL pointer");
    if (n_pts < 0 || n_sun < 0) return fail(SS_ERR_INVALID_ARG, "negative count");
    if (!all_pairs && n_pts != n_sun) return fail(SS_ERR_INVALID_ARG, "paired mode needs n_pts == n_sun");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    SS_HIP(hipSetDevice(m->ctx->device));
    SS_HIP(launch_mlp_prep(w, m->at<uint16_t>(m->L.o_wb), m->at<float>(m->L.o_wf), st));
    const int64_t M = all_pairs ? n_pts * n_sun : n_pts;
    SS_HIP(launch_mlp_forward(m->at<uint16_t>(m->L.o_wb), m->at<float>(m->L.o_wf), pts, sun, M,
                              all_pairs ? n_pts : 0, mlp_norm(m), prob != 0, out, nullptr, nullptr,
                              st));
    return SS_OK;
}

}  // extern "C"

// MLP backward (recomputing forward + BCE / given-logit-gradient adjoint + weight
// gradients) with its buffers at `base` laid out by L (L sized for >= M points).
static ss_status mlp_backward_at(const ss_mlp *m, char *base, const MlpLayout &L, const float *w,
                                 const float *pts, const float *sun, int64_t M,
                                 const float *labels, const float *d_logits, float scale,
                                 float *d_w, float *loss, hipStream_t st)
{
    auto at16 = [base](size_t off) { return reinterpret_cast<uint16_t *>(base + off); };
    auto at32 = [base](size_t off) { return reinterpret_cast<float *>(base + off); };
    uint16_t *wb = at16(L.o_wb);
    float *wf = at32(L.o_wf);
    uint16_t *F = at16(L.o_F);
    uint16_t *H = at16(L.o_H);
    uint16_t *H1 = H, *H2 = H + M * kMlpWidth, *H3 = H + 2 * M * kMlpWidth;
    uint16_t *dA0 = at16(L.o_dA), *dA1 = dA0 + M * kMlpWidth;
    float *logit = at32(L.o_logit);
    float *pdw = at32(L.o_pdw), *pdb = at32(L.o_pdb), *pout = at32(L.o_pout);
    const int nblk = mlp_dw_blocks(M);
    const int nout = (int)((M + 255) / 256);
    SS_HIP(launch_mlp_prep(w, wb, wf, st));
    // saved activations: saveH holds h1, h2, h3 contiguous ([3][M][64])
    SS_HIP(launch_mlp_forward(wb, wf, pts, sun, M, 0, mlp_norm(m), false, logit, F, H, st));
    SS_HIP(launch_mlp_out_bwd(logit, labels, d_logits, scale, wb, H3, M, dA0, pout, st));
    SS_HIP(launch_mlp_reduce(pout, nout, kMlpWidth + 1, 66, d_w + kOffW4, st));
    if (loss) SS_HIP(launch_mlp_reduce(pout + 65, nout, 1, 66, loss, st));
    // layer 3
    SS_HIP(launch_mlp_dw(dA0, H2, kMlpWidth, M, pdw, pdb, st));
    SS_HIP(launch_mlp_reduce(pdw, nblk, kMlpW3, kMlpW3, d_w + kOffW3, st));
    SS_HIP(launch_mlp_reduce(pdb, nblk, kMlpWidth, kMlpWidth, d_w + kOffB3, st));
    SS_HIP(launch_mlp_dh(dA0, wb + kMlpW1 + kMlpW2, H2, M, dA1, st));
    // layer 2
    SS_HIP(launch_mlp_dw(dA1, H1, kMlpWidth, M, pdw, pdb, st));
    SS_HIP(launch_mlp_reduce(pdw, nblk, kMlpW2, kMlpW2, d_w + kOffW2, st));
    SS_HIP(launch_mlp_reduce(pdb, nblk, kMlpWidth, kMlpWidth, d_w + kOffB2, st));
    SS_HIP(launch_mlp_dh(dA1, wb + kMlpW1, H1, M, dA0, st));
    // layer 1
    SS_HIP(launch_mlp_dw(dA0, F, kMlpIn, M, pdw, pdb, st));
    SS_HIP(launch_mlp_reduce(pdw, nblk, kMlpW1, kMlpW1, d_w + kOffW1, st));
    SS_HIP(launch_mlp_reduce(pdb, nblk, kMlpWidth, kMlpWidth, d_w + kOffB1, st));
    return SS_OK;
}

extern "C" {

ss_status ss_mlp_backward(ss_mlp *m, const float *w, const float *pts, const float *sun, int64_t M,
                          const float *labels, const float *d_logits, float scale, float *d_w,
                          float *loss, ss_stream stream)
{
    if (!m || !m->ws) return fail(SS_ERR_STATE, "MLP has no workspace");
    if (!w || !pts || !sun || !d_w || (!labels && !d_logits))
        return fail(SS_ERR_INVALID_ARG, "NULL pointer");
    if (M < 1 || M > m->maxp) return fail(SS_ERR_CAPACITY, "M must be in [1, max_points]");
    SS_HIP(hipSetDevice(m->ctx->device));
    return mlp_backward_at(m, m->ws, m->L, w, pts, sun, M, labels, d_logits, scale, d_w, loss,
                           reinterpret_cast<hipStream_t>(stream));
}

ss_status ss_mlp_backward_noalloc(ss_mlp *m, const float *w, const float *pts, const float *sun,
                                  int64_t M, const float *labels, const float *d_logits,
                                  float scale, float *d_w, float *loss, ss_stream stream)
{
    if (!m || !m->ctx) return fail(SS_ERR_INVALID_ARG, "mlp is NULL");
    if (!w || !pts || !sun || !d_w || (!labels && !d_logits))
        return fail(SS_ERR_INVALID_ARG, "NULL pointer");
    if (M < 1 || M > kNoAllocMaxPoints)
        return fail(SS_ERR_CAPACITY, "M must be in [1, SS_NOALLOC_MAX_POINTS = " +
                                         std::to_string(kNoAllocMaxPoints) + "]");
    if (!m->ctx->scratch) return fail(SS_ERR_STATE, "no scratch array on this device");
    SS_HIP(hipSetDevice(m->ctx->device));
    return mlp_backward_at(m, m->ctx->scratch, kNoAllocLayout, w, pts, sun, M, labels, d_logits,
                           scale, d_w, loss, reinterpret_cast<hipStream_t>(stream));
}

ss_status ss_mlp_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float beta1,
                      float beta2, float eps, int32_t step, ss_stream stream)
{
    if (!w || !m || !v || !g || n < 0 || step < 1) return fail(SS_ERR_INVALID_ARG, "bad arguments");
    SS_HIP(launch_mlp_adam(w, m, v, g, n, lr, beta1, beta2, eps, step,
                           reinterpret_cast<hipStream_t>(stream)));
    return SS_OK;
}

ss_status ss_shadow_surrogate(ss_plan *p, ss_mlp *mlp, const float *w, const ss_surfels *s,
                              const ss_views *v, float band, float *vis, float *sun_depth,
                              ss_stream stream)
{
    ss_status e = check_call(p, s, v);
    if (e != SS_OK) return e;
    if (!mlp || !mlp->ws) return fail(SS_ERR_STATE, "MLP has no workspace");
    if (!v->sun || !vis || !w) return fail(SS_ERR_INVALID_ARG, "views.sun, vis and w are required");
    if (!(band >= 0.f && band <= 0.5f)) return fail(SS_ERR_INVALID_ARG, "band must be in [0, 0.5]");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const Layout &L = p->L;
    p->sun_valid = false;
    unsigned long long *counters = p->at<unsigned long long>(L.counters);
    SS_HIP(fill_u32(p->at<uint32_t>(L.flags) + 1, 0u, 1, st));
    SS_HIP(fill_u32(reinterpret_cast<uint32_t *>(counters + 6), 0u, 2, st));
    unsigned long long *stat = p->at<unsigned long long>(L.stat_sun);
    SS_HIP(fill_u32(reinterpret_cast<uint32_t *>(stat), 0u, 2 * kStatSlots * kStatStride, st));
    {
        StageScope scope(p, SS_STAGE_MLP, st);
        SS_HIP(launch_mlp_prep(w, mlp->at<uint16_t>(mlp->L.o_wb), mlp->at<float>(mlp->L.o_wf), st));
        SS_HIP(launch_mlp_forward(mlp->at<uint16_t>(mlp->L.o_wb), mlp->at<float>(mlp->L.o_wf), s->mean,
                                  v->sun, p->n * (int64_t)p->nv, p->n, mlp_norm(mlp), true, vis,
                                  nullptr, nullptr, st));
    }
    // band 0: no point can fall back, the network's output is the whole pass
    if (band == 0.f) return SS_OK;
    uint32_t *order;
    float *sorted;
    if ((e = prepare(p, s, v, true, &order, &sorted, st)) != SS_OK) return e;
    {
        StageScope scope(p, SS_STAGE_SUN_CAMERA, st);
        SS_HIP(launch_sun_cameras(s->mean, p->n, p->nv, v->Fxy, v->dF, v->sun, v->b_z,
                                  p->st.sun_map_size, p->at<double>(L.bounds),
                                  p->at<SunCam>(L.suncam), st));
    }
    uint32_t *tmask = p->at<uint32_t>(L.tmask_sun);
    {
        StageScope scope(p, SS_STAGE_FALLBACK_FLAG, st);
        SS_HIP(fill_u32(tmask, 0u, p->tiles_sun, st));
        SS_HIP(launch_flag_tiles(s->mean, p->n, p->nv, p->at<SunCam>(L.suncam),
                                 p->at<ViewDesc>(L.views_sun), p->st.sun_map_size, p->st.tile_size,
                                 vis, band, tmask, counters + 6, st));
    }
    if ((e = bin_views(p, v, true, order, sorted, nullptr, true, st, tmask)) != SS_OK) return e;
    float *D = sun_depth ? sun_depth : p->at<float>(L.sun_depth);
    RasterConsts rc = consts(p->st);
    rc.torder = p->torder_sun;
    {
        StageScope scope(p, SS_STAGE_SUN_RASTER, st);
        SS_HIP(launch_raster_fwd(p->st.tile_size, true, false, p->tiles_sun, p->nv,
                                 p->at<ViewDesc>(L.views_sun), p->at<uint32_t>(L.ranges_sun),
                                 p->lists_sun, p->at<float>(L.rec_sun), p->n, rc, nullptr, nullptr,
                                 nullptr, p->at<SunCam>(L.suncam), nullptr, nullptr, nullptr, D,
                                 nullptr, nullptr, nullptr, stat, nullptr, st));
    }
    {
        StageScope scope(p, SS_STAGE_SHADOW_QUERY, st);
        if (band > 0.f)
            SS_HIP(launch_shadow_query(s->mean, p->n, p->nv, p->at<SunCam>(L.suncam), D,
                                       p->st.sun_map_size, v->b_z, p->st.esm_c, p->st.esm_bias, vis,
                                       band, st));
    }
    p->order_sun = order;
    p->sun_order_shared = false;
    p->sun_valid = true;
    return SS_OK;
}

static ss_status adam_args(const ss_adam_config *c, AdamArgs *a)
{
    if (!c || c->struct_size != sizeof(ss_adam_config)) return fail(SS_ERR_INVALID_ARG, "bad ss_adam_config");
    const float lr[7] = {c->lr_mean, c->lr_scale, c->lr_opacity, c->lr_quat, c->lr_albedo, c->lr_dF,
                         c->lr_colour};
    for (int k = 0; k < 7; ++k) {
        if (!(lr[k] >= 0.f) || !std::isfinite(lr[k])) return fail(SS_ERR_INVALID_ARG, "learning rates must be >= 0");
        a->lr[k] = lr[k];
    }
    if (!(c->beta1 >= 0.f && c->beta1 < 1.f) || !(c->beta2 >= 0.f && c->beta2 < 1.f) || !(c->eps >= 0.f))
        return fail(SS_ERR_INVALID_ARG, "Adam betas must be in [0, 1) and eps >= 0");
    a->beta1 = c->beta1; a->beta2 = c->beta2; a->eps = c->eps;
    a->camera_start = c->camera_start;
    return SS_OK;
}

ss_status ss_surfel_activate(int64_t n, const float *raw, float *mean, float *t_u, float *t_v,
                             float *scale, float *opacity, float *albedo, ss_stream stream)
{
    if (n < 0) return fail(SS_ERR_INVALID_ARG, "n < 0");
    if (n > 0 && (!raw || !mean || !t_u || !t_v || !scale || !opacity || !albedo))
        return fail(SS_ERR_INVALID_ARG, "NULL pointer");
    SS_HIP(launch_surfel_activate(n, raw, mean, t_u, t_v, scale, opacity, albedo,
                                  reinterpret_cast<hipStream_t>(stream)));
    return SS_OK;
}

ss_status ss_surfel_raw(int64_t n, const float *mean, const float *t_u, const float *t_v,
                        const float *scale, const float *opacity, const float *albedo, float *raw,
                        ss_stream stream)
{
    if (n < 0) return fail(SS_ERR_INVALID_ARG, "n < 0");
    if (n > 0 && (!raw || !mean || !t_u || !t_v || !scale || !opacity || !albedo))
        return fail(SS_ERR_INVALID_ARG, "NULL pointer");
    SS_HIP(launch_surfel_raw(n, mean, t_u, t_v, scale, opacity, albedo, raw,
                             reinterpret_cast<hipStream_t>(stream)));
    return SS_OK;
}

ss_status ss_adam_surfels(int64_t n, float *raw, float *m, float *v, const float *d_mean,
                          const float *d_t_u, const float *d_t_v, const float *d_scale,
                          const float *d_opacity, const float *d_albedo,
                          const ss_adam_config *cfg, int32_t step, float *mean, float *t_u,
                          float *t_v, float *scale, float *opacity, float *albedo, ss_stream stream)
{
    AdamArgs a;
    ss_status e = adam_args(cfg, &a);
    if (e != SS_OK) return e;
    if (n < 0 || step < 1) return fail(SS_ERR_INVALID_ARG, "n < 0 or step < 1");
    if (n > 0 && (!raw || !m || !v || !d_mean || !d_t_u || !d_t_v || !d_scale || !d_opacity ||
                  !d_albedo || !mean || !t_u || !t_v || !scale || !opacity || !albedo))
        return fail(SS_ERR_INVALID_ARG, "NULL pointer");
    SS_HIP(launch_adam_surfels(n, raw, m, v, d_mean, d_t_u, d_t_v, d_scale, d_opacity, d_albedo, a,
                               step, mean, t_u, t_v, scale, opacity, albedo,
                               reinterpret_cast<hipStream_t>(stream)));
    return SS_OK;
}

ss_status ss_adam_views(int32_t nv, float *dF, float *m_dF, float *v_dF, const float *d_dF,
                        const float *d_dF_extra, float *colC, float *m_colC, float *v_colC, const float *d_colC,
                        float *colc, float *m_colc, float *v_colc, const float *d_colc,
                        const ss_adam_config *cfg, int32_t step, ss_stream stream)
{
    AdamArgs a;
    ss_status e = adam_args(cfg, &a);
    if (e != SS_OK) return e;
    if (nv < 0 || step < 1) return fail(SS_ERR_INVALID_ARG, "nv < 0 or step < 1");
    if ((dF && (!m_dF || !v_dF || !d_dF)) || (colC && (!m_colC || !v_colC || !d_colC)) ||
        (colc && (!m_colc || !v_colc || !d_colc)))
        return fail(SS_ERR_INVALID_ARG, "a parameter group lacks its moments or gradient");
    SS_HIP(launch_adam_views(nv, dF, m_dF, v_dF, d_dF, d_dF_extra, colC, m_colC, v_colC, d_colC, colc, m_colc,
                             v_colc, d_colc, a, step, reinterpret_cast<hipStream_t>(stream)));
    return SS_OK;
}

ss_status ss_image_loss_l1(ss_plan *p, const float *image, const float *target, float weight,
                           float *loss, float *d_image, ss_stream stream)
{
    if (!p) return fail(SS_ERR_INVALID_ARG, "plan is NULL");
    if (!p->ws) return fail(SS_ERR_STATE, "no workspace bound");
    if (!image || !target || !loss || !d_image) return fail(SS_ERR_INVALID_ARG, "NULL pointer");
    if (!std::isfinite(weight)) return fail(SS_ERR_INVALID_ARG, "weight must be finite");
    SS_HIP(hipSetDevice(p->ctx->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    StageScope scope(p, SS_STAGE_IMAGE_LOSS, st);
    SS_HIP(launch_l1_loss(p->at<ViewDesc>(p->L.views_main), p->nv, max_view_pixels(p), image, target,
                          weight, d_image, p->at<double>(p->L.geom_parts), loss, st));
    return SS_OK;
}

ss_status ss_dsm_init_workspace_size(int32_t nx, int32_t ny, size_t *bytes)
{
    if (!bytes || nx < 2 || ny < 2) return fail(SS_ERR_INVALID_ARG, "the DSM needs at least 2 x 2 nodes");
    *bytes = dsm_init_workspace_bytes(nx, ny);
    return SS_OK;
}

ss_status ss_dsm_init(int32_t nx, int32_t ny, const float *z, float x0, float y0, float gsd,
                      int64_t n, uint64_t seed, float opacity, float albedo, void *workspace,
                      size_t bytes, float *mean, float *t_u, float *t_v, float *scale,
                      float *opacity_out, float *albedo_out, int64_t *cell, ss_stream stream)
{
    if (nx < 2 || ny < 2 || !z) return fail(SS_ERR_INVALID_ARG, "the DSM needs at least 2 x 2 nodes");
    if ((int64_t)(nx - 1) * (int64_t)(ny - 1) > (int64_t(1) << 36))
        return fail(SS_ERR_UNSUPPORTED, "DSM too large");
    if (!(gsd > 0.f) || !std::isfinite(gsd) || !std::isfinite(x0) || !std::isfinite(y0))
        return fail(SS_ERR_INVALID_ARG, "gsd must be positive, the origin finite");
    if (n < 0 || n > (int64_t(1) << 32)) return fail(SS_ERR_INVALID_ARG, "n must be in [0, 2^32]");
    if (!workspace || bytes < dsm_init_workspace_bytes(nx, ny) || ((uintptr_t)workspace & 255))
        return fail(SS_ERR_CAPACITY, "workspace missing, unaligned or smaller than ss_dsm_init_workspace_size");
    if (n > 0 && (!mean || !t_u || !t_v || !scale || !opacity_out || !albedo_out))
        return fail(SS_ERR_INVALID_ARG, "NULL output");
    SS_HIP(launch_dsm_init(nx, ny, z, (double)x0, (double)y0, (double)gsd, n, seed, opacity, albedo,
                           workspace, mean, t_u, t_v, scale, opacity_out, albedo_out, cell,
                           reinterpret_cast<hipStream_t>(stream)));
    return SS_OK;
}

static const char *kStageNames[SS_NUM_STAGES] = {
    "depth_sort", "project", "bin", "raster_fwd", "raster_bwd", "project_bwd", "reduce",
    "sun_camera", "sun_project", "sun_bin", "sun_raster", "shadow_query", "mlp_forward",
    "fallback_flag", "normal_loss", "image_loss"};

const char *ss_stage_name(int32_t stage)
{
    return (stage >= 0 && stage < SS_NUM_STAGES) ? kStageNames[stage] : "";
}

ss_status ss_plan_set_timing(ss_plan *p, int32_t enable)
{
    if (!p) return fail(SS_ERR_INVALID_ARG, "plan is NULL");
    p->timer.on = enable != 0;
    return SS_OK;
}

ss_status ss_plan_read_timing(ss_plan *p, double *ms, int64_t *launches)
{
    if (!p) return fail(SS_ERR_INVALID_ARG, "plan is NULL");
    StageTimer &t = p->timer;
    if (!t.pending.empty()) SS_HIP(hipEventSynchronize(t.pending.back().b));
    for (const auto &q : t.pending) {
        float e = 0.f;
        SS_HIP(hipEventElapsedTime(&e, q.a, q.b));
        t.ms[q.stage] += e;
        t.count[q.stage] += 1;
    }
    t.pending.clear();
    t.used = 0;
    for (int k = 0; k < SS_NUM_STAGES; ++k) {
        if (ms) ms[k] = t.ms[k];
        if (launches) launches[k] = t.count[k];
        t.ms[k] = 0.0;
        t.count[k] = 0;
    }
    return SS_OK;
}

ss_status ss_plan_stats(ss_plan *p, int64_t *out, ss_stream stream)
{
    if (!p || !p->ws || !out) return fail(SS_ERR_INVALID_ARG, "plan/workspace/out missing");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    unsigned long long c[7];
    std::vector<unsigned long long> sm((size_t)kStatSlots * kStatStride), ss((size_t)kStatSlots * kStatStride);
    SS_HIP(hipMemcpyAsync(c, p->at<void>(p->L.counters), sizeof c, hipMemcpyDeviceToHost, st));
    SS_HIP(hipMemcpyAsync(sm.data(), p->at<void>(p->L.stat_main), sm.size() * 8, hipMemcpyDeviceToHost, st));
    SS_HIP(hipMemcpyAsync(ss.data(), p->at<void>(p->L.stat_sun), ss.size() * 8, hipMemcpyDeviceToHost, st));
    SS_HIP(hipStreamSynchronize(st));
    // pairs main, contributing main, evaluated main, pairs sun, contributing sun, evaluated
    // sun, surrogate fallback points
    for (int k = 2; k < 6; ++k) c[k] = 0;
    for (int q = 0; q < kStatSlots; ++q) {
        c[2] += sm[(size_t)q * kStatStride]; c[3] += sm[(size_t)q * kStatStride + 1];
        c[4] += ss[(size_t)q * kStatStride]; c[5] += ss[(size_t)q * kStatStride + 1];
    }
    const int map[7] = {0, 2, 3, 1, 4, 5, 6};
    for (int k = 0; k < 7; ++k) out[k] = (int64_t)c[map[k]];
    return SS_OK;
}

}  // extern "C"

// C ABI of the rasterizer (declared in include/h4dgs.h): argument checks,
// workspace layout and the launch sequence of each entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/h4dgs.h"
#include "common.hpp"
#include "launch.hpp"

struct h4d_ctx {
    std::string err;
};

namespace h4d {
namespace {

h4d_status fail(h4d_ctx* c, h4d_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

h4d_status hip_check(h4d_ctx* c, const char* where) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, H4D_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
    return H4D_OK;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    }
};

struct ViewGeom {
    int tiles_x, tiles_y, tile_base;
    int64_t pix_base;
};

struct Layout {
    int N = 0, V = 0, total_tiles = 0;
    int64_t total_pix = 0;
    uint64_t cap = 0;
    ViewGeom vg[kMaxViews];
    // state
    size_t st_status, st_pair_base, st_views, st_recs, st_ids, st_ranges, st_T, st_nc, st_C, state_bytes;
    // scratch, forward use
    size_t sc_dkeys, sc_dvals, sc_dkeys2, sc_dvals2, sc_ntiles, sc_offsets, sc_partials, sc_eff, sc_pkeys, sc_pvals,
        sc_pkeys2, sc_pvals2, sc_hist, sc_totals, fwd_bytes;
    // scratch, backward use
    size_t sc_g2, bwd_bytes;
    size_t scratch_bytes;
};

Layout make_layout(int N, const h4d_view* views, int V, const h4d_config* cfg) {
    Layout L;
    L.N = N;
    L.V = V;
    L.cap = (uint64_t)std::max<int64_t>(0, cfg->pair_capacity);
    int tb = 0;
    int64_t pb = 0;
    for (int v = 0; v < V; ++v) {
        L.vg[v].tiles_x = ceil_div(views[v].width, cfg->tile);
        L.vg[v].tiles_y = ceil_div(views[v].height, cfg->tile);
        L.vg[v].tile_base = tb;
        L.vg[v].pix_base = pb;
        tb += L.vg[v].tiles_x * L.vg[v].tiles_y;
        pb += (int64_t)views[v].width * views[v].height;
    }
    L.total_tiles = tb;
    L.total_pix = pb;
    const size_t n = (size_t)N, V_ = (size_t)V;
    Carve s;
    L.st_status = s.take(sizeof(Status));
    L.st_pair_base = s.take(8 * (V_ + 1));
    L.st_views = s.take(sizeof(ViewParams) * V_);
    L.st_recs = s.take(sizeof(Rec) * n * V_);
    L.st_ids = s.take(4 * (size_t)L.cap);
    L.st_ranges = s.take(16 * (size_t)tb);
    L.st_T = s.take(4 * (size_t)pb);
    L.st_nc = s.take(4 * (size_t)pb);
    L.st_C = s.take(12 * (size_t)pb);
    L.state_bytes = s.off;
    Carve f;
    L.sc_dkeys = f.take(4 * n);
    L.sc_dvals = f.take(4 * n);
    L.sc_dkeys2 = f.take(4 * n);
    L.sc_dvals2 = f.take(4 * n);
    L.sc_ntiles = f.take(4 * n);
    L.sc_offsets = f.take(8 * (n + 1));
    L.sc_partials = f.take(8 * ((size_t)scan_blocks(N) + 2));
    L.sc_eff = f.take(8);
    L.sc_pkeys = f.take(4 * (size_t)L.cap);
    L.sc_pvals = f.take(4 * (size_t)L.cap);
    L.sc_pkeys2 = f.take(4 * (size_t)L.cap);
    L.sc_pvals2 = f.take(4 * (size_t)L.cap);
    L.sc_hist = f.take(4 * radix_hist_words(std::max<uint64_t>(L.cap, n)));
    L.sc_totals = f.take(4 * 256);
    L.fwd_bytes = f.off;
    Carve b;
    L.sc_g2 = b.take(4 * 9 * n * V_);
    L.bwd_bytes = b.off;
    L.scratch_bytes = std::max(L.fwd_bytes, L.bwd_bytes);
    return L;
}

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

h4d_status check_config(h4d_ctx* c, const h4d_config* cfg) {
    if (!cfg) return fail(c, H4D_ERR_INVALID_ARG, "config is null");
    if (!composite_supported(cfg->tile, cfg->chunk))
        return fail(c, H4D_ERR_INVALID_ARG, "tile must be 8, 16 or 32 and chunk 128, 256 or 512 (got %d, %d)",
                    cfg->tile, cfg->chunk);
    if (cfg->pair_capacity < 0) return fail(c, H4D_ERR_INVALID_ARG, "pair_capacity < 0");
    if (cfg->pair_capacity > (int64_t)0xFFFFFFFFll * 4)
        return fail(c, H4D_ERR_INVALID_ARG, "pair_capacity too large");
    if (cfg->batched != 0 && cfg->batched != 1) return fail(c, H4D_ERR_INVALID_ARG, "batched must be 0 or 1");
    return H4D_OK;
}

h4d_status check_views(h4d_ctx* c, const h4d_view* views, int n_views) {
    if (!views) return fail(c, H4D_ERR_INVALID_ARG, "views is null");
    if (n_views < 1 || n_views > kMaxViews)
        return fail(c, H4D_ERR_INVALID_ARG, "n_views must be in [1, %d] (got %d)", kMaxViews, n_views);
    for (int v = 0; v < n_views; ++v) {
        const h4d_view& w = views[v];
        if (w.width < 1 || w.height < 1 || w.width > 32767 || w.height > 32767)
            return fail(c, H4D_ERR_INVALID_ARG, "view %d: image size %dx%d outside [1, 32767]", v, w.width, w.height);
        if (!(w.fx > 0.f) || !(w.fy > 0.f) || !std::isfinite(w.fx) || !std::isfinite(w.fy))
            return fail(c, H4D_ERR_INVALID_ARG, "view %d: focal lengths must be finite and > 0", v);
        for (int k = 0; k < 12; ++k)
            if (!std::isfinite(w.world_to_cam[k])) return fail(c, H4D_ERR_INVALID_ARG, "view %d: non-finite pose", v);
        if (!std::isfinite(w.t) || !std::isfinite(w.cx) || !std::isfinite(w.cy))
            return fail(c, H4D_ERR_INVALID_ARG, "view %d: non-finite t / principal point", v);
    }
    return H4D_OK;
}

h4d_status check_sets(h4d_ctx* c, const h4d_g3d* g3, const h4d_g4d* g4) {
    if (!g3 || !g4) return fail(c, H4D_ERR_INVALID_ARG, "Gaussian set descriptor is null");
    if (g3->n < 0 || g4->n < 0) return fail(c, H4D_ERR_INVALID_ARG, "negative Gaussian count");
    if ((int64_t)g3->n + g4->n > (int64_t)0x7FFFFFFF) return fail(c, H4D_ERR_INVALID_ARG, "too many Gaussians");
    if (g3->n > 0 && (!g3->mean || !g3->log_scale || !g3->quat || !g3->opacity || !g3->sh))
        return fail(c, H4D_ERR_INVALID_ARG, "3D set: null array with n = %d", g3->n);
    if (g4->n > 0 && (!g4->mean || !g4->mean_t || !g4->log_scale || !g4->quat_l || !g4->quat_r || !g4->opacity ||
                      !g4->sh))
        return fail(c, H4D_ERR_INVALID_ARG, "4D set: null array with n = %d", g4->n);
    return H4D_OK;
}

G3Ptr to_ptr(const h4d_g3d* g) { return G3Ptr{g->n, g->mean, g->log_scale, g->quat, g->opacity, g->sh}; }
G4Ptr to_ptr(const h4d_g4d* g) {
    return G4Ptr{g->n, g->mean, g->mean_t, g->log_scale, g->quat_l, g->quat_r, g->opacity, g->sh};
}

ViewTableIn view_table(const h4d_view* views, int V, int tile) {
    ViewTableIn t;
    std::memset(&t, 0, sizeof(t));
    t.n = V;
    t.tile = tile;
    for (int v = 0; v < V; ++v) {
        ViewIn& o = t.v[v];
        std::memcpy(o.M, views[v].world_to_cam, sizeof(o.M));
        o.fx = views[v].fx; o.fy = views[v].fy; o.cx = views[v].cx; o.cy = views[v].cy;
        o.W = views[v].width; o.H = views[v].height; o.t = views[v].t;
        for (int k = 0; k < 3; ++k) o.bg[k] = views[v].bg[k];
    }
    return t;
}

int bits_for(int tiles) {
    int b = 1;
    while ((1ll << b) < (long long)tiles) ++b;
    return b;
}

// Binning, sorting and blending of one view whose records are in place
// (recs_v, ntiles, dkeys, dvals filled): Alg. 1 lines 7-17.
void bin_and_blend(const Layout& L, int v, int tile, int chunk, void* state, void* scratch, const Rec* recs_v,
                   float* image, hipStream_t st) {
    const int N = L.N;
    uint32_t* dk = at<uint32_t>(scratch, L.sc_dkeys);
    uint32_t* dv = at<uint32_t>(scratch, L.sc_dvals);
    uint32_t* dk2 = at<uint32_t>(scratch, L.sc_dkeys2);
    uint32_t* dv2 = at<uint32_t>(scratch, L.sc_dvals2);
    uint32_t* hist = at<uint32_t>(scratch, L.sc_hist);
    uint32_t* totals = at<uint32_t>(scratch, L.sc_totals);
    // depth order over the Gaussians: 4 stable 8-bit passes over the float32 depth bits
    for (int pass = 0; pass < 4; ++pass) {
        const bool even = (pass % 2) == 0;
        launch_radix_pass(even ? dk : dk2, even ? dv : dv2, even ? dk2 : dk, even ? dv2 : dv, nullptr, (uint64_t)N,
                          (uint64_t)N, 8 * pass, 8, hist, totals, nullptr, st);
    }
    // per depth-ordered Gaussian: offsets of its (Gaussian, tile) pairs
    unsigned long long* offsets = at<unsigned long long>(scratch, L.sc_offsets);
    unsigned long long* partials = at<unsigned long long>(scratch, L.sc_partials);
    unsigned long long* eff = at<unsigned long long>(scratch, L.sc_eff);
    uint32_t* ntiles = at<uint32_t>(scratch, L.sc_ntiles);
    launch_scan_u32_u64(ntiles, dv, N, offsets, partials, st);
    Status* status = at<Status>(state, L.st_status);
    unsigned long long* pair_base = at<unsigned long long>(state, L.st_pair_base);
    launch_finalize_pairs(offsets, N, pair_base, v, L.cap, status, eff, st);
    uint32_t* pk = at<uint32_t>(scratch, L.sc_pkeys);
    uint32_t* pv = at<uint32_t>(scratch, L.sc_pvals);
    uint32_t* pk2 = at<uint32_t>(scratch, L.sc_pkeys2);
    uint32_t* pv2 = at<uint32_t>(scratch, L.sc_pvals2);
    const ViewGeom& g = L.vg[v];
    launch_emit(dv, offsets, N, recs_v, tile, g.tiles_x, eff, pk, pv, st);
    // stable sort of the tile ids; the last pass writes the ids to their final place
    const int tiles = g.tiles_x * g.tiles_y;
    const int bits = bits_for(tiles);
    const int passes = (bits + 7) / 8;
    uint32_t* ids = at<uint32_t>(state, L.st_ids);
    uint32_t* kin = pk;
    uint32_t* vin = pv;
    int shift = 0;
    for (int p = 0; p < passes; ++p) {
        const int nb = (bits - shift + (passes - p) - 1) / (passes - p);
        const bool last = p == passes - 1;
        uint32_t* kout = (kin == pk) ? pk2 : pk;
        uint32_t* vout = last ? ids : ((vin == pv) ? pv2 : pv);
        launch_radix_pass(kin, vin, kout, vout, eff, 0, L.cap, shift, nb, hist, totals, last ? pair_base + v : nullptr,
                          st);
        kin = kout;
        vin = vout;
        shift += nb;
    }
    int64_t* ranges = at<int64_t>(state, L.st_ranges) + 2 * (size_t)g.tile_base;
    launch_ranges(kin, eff, pair_base + v, ranges, st);
    const ViewParams* vp = at<ViewParams>(state, L.st_views);
    launch_composite_fwd(tile, chunk, recs_v, ids, at<int64_t>(state, L.st_ranges), vp, v, tiles, image,
                         at<float>(state, L.st_T), at<uint32_t>(state, L.st_nc), at<float>(state, L.st_C), st);
}

}  // namespace
}  // namespace h4d

using namespace h4d;

extern "C" {

const char* h4dgs_version(void) { return "h4dgs 0.1 (gfx950)"; }

h4d_status h4dgs_create(h4d_ctx** out) {
    if (!out) return H4D_ERR_INVALID_ARG;
    *out = new (std::nothrow) h4d_ctx();
    return *out ? H4D_OK : H4D_ERR_INVALID_ARG;
}

h4d_status h4dgs_destroy(h4d_ctx* ctx) {
    delete ctx;
    return H4D_OK;
}

const char* h4dgs_last_error(const h4d_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

h4d_status h4dgs_workspace_size(h4d_ctx* ctx, int32_t n3, int32_t n4, const h4d_view* views, int32_t n_views,
                                const h4d_config* cfg, size_t* state_bytes, size_t* scratch_bytes) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_config(ctx, cfg)) != H4D_OK) return s;
    if ((s = check_views(ctx, views, n_views)) != H4D_OK) return s;
    if (n3 < 0 || n4 < 0 || (int64_t)n3 + n4 > 0x7FFFFFFF) return fail(ctx, H4D_ERR_INVALID_ARG, "bad Gaussian counts");
    if (!state_bytes || !scratch_bytes) return fail(ctx, H4D_ERR_INVALID_ARG, "null size output");
    const Layout L = make_layout(n3 + n4, views, n_views, cfg);
    *state_bytes = L.state_bytes;
    *scratch_bytes = L.scratch_bytes;
    return H4D_OK;
}

h4d_status h4dgs_render_fwd(h4d_ctx* ctx, const h4d_g3d* g3, const h4d_g4d* g4, const h4d_view* views,
                            int32_t n_views, const h4d_config* cfg, float* const* images, void* state,
                            size_t state_bytes, void* scratch, size_t scratch_bytes, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_sets(ctx, g3, g4)) != H4D_OK) return s;
    if ((s = check_config(ctx, cfg)) != H4D_OK) return s;
    if ((s = check_views(ctx, views, n_views)) != H4D_OK) return s;
    if (cfg->batched) return fail(ctx, H4D_ERR_UNSUPPORTED, "batched mode is not available in this build");
    if (!images) return fail(ctx, H4D_ERR_INVALID_ARG, "images is null");
    for (int v = 0; v < n_views; ++v)
        if (!images[v]) return fail(ctx, H4D_ERR_INVALID_ARG, "image %d is null", v);
    const int N = g3->n + g4->n;
    const Layout L = make_layout(N, views, n_views, cfg);
    if (!state || state_bytes < L.state_bytes)
        return fail(ctx, H4D_ERR_INVALID_ARG, "state too small (%zu < %zu)", state_bytes, L.state_bytes);
    if (!scratch || scratch_bytes < L.fwd_bytes)
        return fail(ctx, H4D_ERR_INVALID_ARG, "scratch too small (%zu < %zu)", scratch_bytes, L.fwd_bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const G3Ptr p3 = to_ptr(g3);
    const G4Ptr p4 = to_ptr(g4);
    ViewParams* vp = at<ViewParams>(state, L.st_views);
    launch_write_views(view_table(views, n_views, cfg->tile), vp, st);
    launch_zero_status(at<Status>(state, L.st_status), at<unsigned long long>(state, L.st_pair_base), n_views, st);
    launch_fill_u64(at<unsigned long long>(state, L.st_ranges), 2 * (size_t)L.total_tiles, 0ull, st);
    for (int v = 0; v < n_views; ++v) {
        Rec* recs_v = at<Rec>(state, L.st_recs) + (size_t)v * N;
        launch_preprocess(p3, p4, vp, v, cfg->tile, recs_v, at<uint32_t>(scratch, L.sc_ntiles),
                          at<uint32_t>(scratch, L.sc_dkeys), at<uint32_t>(scratch, L.sc_dvals), st);
        bin_and_blend(L, v, cfg->tile, cfg->chunk, state, scratch, recs_v, images[v], st);
    }
    return hip_check(ctx, "render_fwd");
}

h4d_status h4dgs_render_bwd(h4d_ctx* ctx, const h4d_g3d* g3, const h4d_g4d* g4, const h4d_view* views,
                            int32_t n_views, const h4d_config* cfg, const float* const* dl_dimages, const void* state,
                            size_t state_bytes, void* scratch, size_t scratch_bytes, h4d_g3d_mut* grad3,
                            h4d_g4d_mut* grad4, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_sets(ctx, g3, g4)) != H4D_OK) return s;
    if ((s = check_config(ctx, cfg)) != H4D_OK) return s;
    if ((s = check_views(ctx, views, n_views)) != H4D_OK) return s;
    if (cfg->batched) return fail(ctx, H4D_ERR_UNSUPPORTED, "batched mode is not available in this build");
    if (!dl_dimages) return fail(ctx, H4D_ERR_INVALID_ARG, "dl_dimages is null");
    for (int v = 0; v < n_views; ++v)
        if (!dl_dimages[v]) return fail(ctx, H4D_ERR_INVALID_ARG, "dl_dimage %d is null", v);
    if (!grad3 || !grad4) return fail(ctx, H4D_ERR_INVALID_ARG, "gradient descriptor is null");
    if (grad3->n != g3->n || grad4->n != g4->n) return fail(ctx, H4D_ERR_INVALID_ARG, "gradient counts differ");
    if (g3->n > 0 && (!grad3->mean || !grad3->log_scale || !grad3->quat || !grad3->opacity || !grad3->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "3D gradient: null array");
    if (g4->n > 0 && (!grad4->mean || !grad4->mean_t || !grad4->log_scale || !grad4->quat_l || !grad4->quat_r ||
                      !grad4->opacity || !grad4->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "4D gradient: null array");
    const int N = g3->n + g4->n;
    const Layout L = make_layout(N, views, n_views, cfg);
    if (!state || state_bytes < L.state_bytes)
        return fail(ctx, H4D_ERR_INVALID_ARG, "state too small (%zu < %zu)", state_bytes, L.state_bytes);
    if (!scratch || scratch_bytes < L.bwd_bytes)
        return fail(ctx, H4D_ERR_INVALID_ARG, "scratch too small (%zu < %zu)", scratch_bytes, L.bwd_bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    void* stt = const_cast<void*>(state);
    float* g2 = at<float>(scratch, L.sc_g2);
    launch_fill_f32(g2, (size_t)9 * N * n_views, 0.f, st);
    const ViewParams* vp = at<ViewParams>(stt, L.st_views);
    for (int v = 0; v < n_views; ++v) {
        const int tiles = L.vg[v].tiles_x * L.vg[v].tiles_y;
        launch_composite_bwd(cfg->tile, cfg->chunk, at<Rec>(stt, L.st_recs) + (size_t)v * N, at<uint32_t>(stt, L.st_ids),
                             at<int64_t>(stt, L.st_ranges), vp, v, tiles, dl_dimages[v], at<float>(stt, L.st_T),
                             at<uint32_t>(stt, L.st_nc), at<float>(stt, L.st_C), g2 + (size_t)v * 9 * N, N, st);
    }
    const G3Grad r3{grad3->n, grad3->mean, grad3->log_scale, grad3->quat, grad3->opacity, grad3->sh};
    const G4Grad r4{grad4->n, grad4->mean, grad4->mean_t, grad4->log_scale, grad4->quat_l, grad4->quat_r,
                    grad4->opacity, grad4->sh};
    launch_preprocess_bwd(to_ptr(g3), to_ptr(g4), vp, n_views, at<Rec>(stt, L.st_recs), g2, r3, r4, st);
    return hip_check(ctx, "render_bwd");
}

h4d_status h4dgs_check(h4d_ctx* ctx, const void* state, size_t state_bytes, int64_t* pairs_needed, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    if (!state || state_bytes < sizeof(Status)) return fail(ctx, H4D_ERR_INVALID_ARG, "state too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(st) != hipSuccess) return hip_check(ctx, "check: stream synchronize");
    Status hs;
    if (hipMemcpy(&hs, state, sizeof(Status), hipMemcpyDeviceToHost) != hipSuccess)
        return hip_check(ctx, "check: status copy");
    if (pairs_needed) *pairs_needed = (int64_t)hs.pairs_needed;
    if (hs.flags & kFlagOverflow)
        return fail(ctx, H4D_ERR_CAPACITY, "pair capacity exceeded: %llu pairs needed", hs.pairs_needed);
    return H4D_OK;
}

h4d_status h4dgs_rasterize_splats(h4d_ctx* ctx, int32_t n, const float* u, const float* v, const float* conic,
                                  const float* opacity, const float* rgb, const int32_t* radius, const float* depth,
                                  const uint8_t* visible, int32_t width, int32_t height, const float* bg,
                                  const h4d_config* cfg, float* image, float* T_final, uint32_t* sorted_ids,
                                  int64_t* ranges, void* state, size_t state_bytes, void* scratch,
                                  size_t scratch_bytes, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_config(ctx, cfg)) != H4D_OK) return s;
    if (cfg->batched) return fail(ctx, H4D_ERR_UNSUPPORTED, "batched mode is not available in this build");
    if (n < 0) return fail(ctx, H4D_ERR_INVALID_ARG, "n < 0");
    if (n > 0 && (!u || !v || !conic || !opacity || !rgb || !radius || !depth || !visible))
        return fail(ctx, H4D_ERR_INVALID_ARG, "null splat array");
    if (!image || !bg) return fail(ctx, H4D_ERR_INVALID_ARG, "image / bg is null");
    h4d_view view;
    std::memset(&view, 0, sizeof(view));
    view.world_to_cam[0] = view.world_to_cam[5] = view.world_to_cam[10] = 1.f;
    view.fx = view.fy = 1.f;
    view.width = width;
    view.height = height;
    for (int k = 0; k < 3; ++k) view.bg[k] = bg[k];
    if ((s = check_views(ctx, &view, 1)) != H4D_OK) return s;
    const Layout L = make_layout(n, &view, 1, cfg);
    if (!state || state_bytes < L.state_bytes) return fail(ctx, H4D_ERR_INVALID_ARG, "state too small");
    if (!scratch || scratch_bytes < L.fwd_bytes) return fail(ctx, H4D_ERR_INVALID_ARG, "scratch too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_write_views(view_table(&view, 1, cfg->tile), at<ViewParams>(state, L.st_views), st);
    launch_zero_status(at<Status>(state, L.st_status), at<unsigned long long>(state, L.st_pair_base), 1, st);
    launch_fill_u64(at<unsigned long long>(state, L.st_ranges), 2 * (size_t)L.total_tiles, 0ull, st);
    Rec* recs = at<Rec>(state, L.st_recs);
    launch_splats_to_records(n, u, v, conic, opacity, rgb, radius, depth, visible, width, height, cfg->tile, recs,
                             at<uint32_t>(scratch, L.sc_ntiles), at<uint32_t>(scratch, L.sc_dkeys),
                             at<uint32_t>(scratch, L.sc_dvals), st);
    bin_and_blend(L, 0, cfg->tile, cfg->chunk, state, scratch, recs, image, st);
    const size_t hw = (size_t)width * height;
    if (T_final) (void)hipMemcpyAsync(T_final, at<float>(state, L.st_T), 4 * hw, hipMemcpyDeviceToDevice, st);
    if (sorted_ids && L.cap > 0)
        (void)hipMemcpyAsync(sorted_ids, at<uint32_t>(state, L.st_ids), 4 * (size_t)L.cap, hipMemcpyDeviceToDevice, st);
    if (ranges)
        (void)hipMemcpyAsync(ranges, at<int64_t>(state, L.st_ranges), 16 * (size_t)L.total_tiles,
                             hipMemcpyDeviceToDevice, st);
    return hip_check(ctx, "rasterize_splats");
}

size_t h4dgs_convert_scratch_bytes(int32_t n4) {
    const size_t n = (size_t)std::max(0, n4);
    const size_t nb = (size_t)std::max(1, scan_blocks(n4));
    return align_up(8 * n) + align_up(16 * (n + 1)) + align_up(16 * (nb + 1)) + align_up(16);
}

h4d_status h4dgs_convert_static(h4d_ctx* ctx, const h4d_g4d* in4, const h4d_g3d* in3, float tau, h4d_g4d_mut* out4,
                                h4d_g3d_mut* out3, int32_t* perm, int32_t* n4_out, int32_t* n3_out, void* scratch,
                                size_t scratch_bytes, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_sets(ctx, in3, in4)) != H4D_OK) return s;
    if (!out4 || !out3 || !n4_out || !n3_out) return fail(ctx, H4D_ERR_INVALID_ARG, "null output");
    if (!(tau > 0.f) || !std::isfinite(tau)) return fail(ctx, H4D_ERR_INVALID_ARG, "tau must be finite and > 0");
    if (out4->n < in4->n) return fail(ctx, H4D_ERR_CAPACITY, "out4 capacity %d < %d", out4->n, in4->n);
    if ((int64_t)out3->n < (int64_t)in3->n + in4->n)
        return fail(ctx, H4D_ERR_CAPACITY, "out3 capacity %d < %d", out3->n, in3->n + in4->n);
    if (in4->n > 0 && (!perm || !out4->mean || !out4->mean_t || !out4->log_scale || !out4->quat_l || !out4->quat_r ||
                       !out4->opacity || !out4->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "null 4D output array");
    if (out3->n > 0 && (!out3->mean || !out3->log_scale || !out3->quat || !out3->opacity || !out3->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "null 3D output array");
    if ((const void*)out3->mean == (const void*)in3->mean || (const void*)out4->mean == (const void*)in4->mean)
        return fail(ctx, H4D_ERR_INVALID_ARG, "outputs must not alias inputs");
    const int n4 = in4->n;
    const size_t need = h4dgs_convert_scratch_bytes(n4);
    if (!scratch || scratch_bytes < need) return fail(ctx, H4D_ERR_INVALID_ARG, "scratch too small (%zu < %zu)",
                                                     scratch_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)n4;
    const size_t nb = (size_t)std::max(1, scan_blocks(n4));
    Carve c;
    const size_t o_flags = c.take(8 * n), o_scan = c.take(16 * (n + 1)), o_part = c.take(16 * (nb + 1)),
                 o_cnt = c.take(16);
    const G4Grad o4{out4->n, out4->mean, out4->mean_t, out4->log_scale, out4->quat_l, out4->quat_r, out4->opacity,
                    out4->sh};
    const G3Grad o3{out3->n, out3->mean, out3->log_scale, out3->quat, out3->opacity, out3->sh};
    const double log_tau = std::log((double)tau);
    int32_t* dcounts = at<int32_t>(scratch, o_cnt);
    launch_convert_static(to_ptr(in4), to_ptr(in3), log_tau, o4, o3, perm, at<uint32_t>(scratch, o_flags),
                          at<unsigned long long>(scratch, o_scan), at<unsigned long long>(scratch, o_part), dcounts,
                          st);
    if ((s = hip_check(ctx, "convert_static")) != H4D_OK) return s;
    int32_t hc[2] = {0, 0};
    if (hipMemcpyAsync(hc, dcounts, sizeof(hc), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return hip_check(ctx, "convert_static: count readback");
    *n4_out = hc[0];
    *n3_out = hc[1];
    return H4D_OK;
}

h4d_status h4dgs_adam(h4d_ctx* ctx, int32_t n_seg, float* const* params, const float* const* grads, float* const* m,
                      float* const* v, const int64_t* sizes, const float* lrs, float beta1, float beta2, float eps,
                      int32_t step, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    if (n_seg < 0 || n_seg > kMaxAdamSeg)
        return fail(ctx, H4D_ERR_INVALID_ARG, "n_seg must be in [0, %d]", kMaxAdamSeg);
    if (n_seg > 0 && (!params || !grads || !m || !v || !sizes || !lrs))
        return fail(ctx, H4D_ERR_INVALID_ARG, "null segment table");
    if (step < 1) return fail(ctx, H4D_ERR_INVALID_ARG, "step must be >= 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
        return fail(ctx, H4D_ERR_INVALID_ARG, "bad Adam constants");
    AdamTable t;
    std::memset(&t, 0, sizeof(t));
    t.n_seg = n_seg;
    t.b1 = beta1; t.b2 = beta2; t.eps = eps;
    t.c1 = (float)(1.0 - std::pow((double)beta1, step));
    t.c2 = (float)(1.0 - std::pow((double)beta2, step));
    for (int i = 0; i < n_seg; ++i) {
        if (sizes[i] < 0) return fail(ctx, H4D_ERR_INVALID_ARG, "segment %d: negative size", i);
        if (sizes[i] > 0 && (!params[i] || !grads[i] || !m[i] || !v[i]))
            return fail(ctx, H4D_ERR_INVALID_ARG, "segment %d: null pointer", i);
        t.seg[i] = AdamSeg{params[i], grads[i], m[i], v[i], sizes[i], lrs[i]};
    }
    launch_adam(t, static_cast<hipStream_t>(stream));
    return hip_check(ctx, "adam");
}

}  // extern "C"

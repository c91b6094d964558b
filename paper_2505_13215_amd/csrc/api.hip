// C ABI of the rasterizer (declared in include/h4dgs.h): argument checks,
// workspace layout and the launch sequence of each entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/h4dgs.h"
#include "common.hpp"
#include "launch.hpp"

struct h4d_ctx {
    std::string err;
    // 0 off, 1 stages bracketed by events, 2 both blending kernels by their own
    // timestamps, 3 the forward one only, 4 the backward one only
    int profile = 0;
    bool stats = false;
    struct Mark {
        hipEvent_t a, b;
        int stage;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Mark> marks;
    hipEvent_t event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~h4d_ctx() {
        for (auto& m : marks) {
            if (m.a) (void)hipEventDestroy(m.a);
            if (m.b) (void)hipEventDestroy(m.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// Workspace of h4dgs_render_infer_noalloc (state and scratch of one call), for
// callers that cannot allocate.  Every GPU the library runs on holds its own
// copy at its own address until the process ends.  Host code never uses this
// name as an address: it asks hipGetSymbolAddress for the current device's
// copy once and passes that pointer on.
static __device__ __align__(256) unsigned char noalloc_workspace[H4DGS_NOALLOC_BYTES];

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

// Brackets one stage's launches with events when profiling is enabled.
struct StageScope {
    h4d_ctx* c;
    hipStream_t st;
    int stage;
    hipEvent_t a = nullptr;
    StageScope(h4d_ctx* c_, hipStream_t st_, int stage_) : c(c_), st(st_), stage(stage_) {
        if (c && c->profile == 1) {
            a = c->event();
            if (a) (void)hipEventRecord(a, st);
        }
    }
    ~StageScope() {
        if (c && a) {
            hipEvent_t b = c->event();
            if (b) {
                (void)hipEventRecord(b, st);
                c->marks.push_back(h4d_ctx::Mark{a, b, stage});
            } else {
                c->pool.push_back(a);
            }
        }
    }
};

// Events for one blend launch timed from its own dispatch (profile levels 2-4);
// both null otherwise.  The launch must happen (non-empty grid).
struct KernelMark {
    h4d_ctx* c;
    int stage;
    hipEvent_t a = nullptr, b = nullptr;
    KernelMark(h4d_ctx* c_, int stage_, bool launches) : c(c_), stage(stage_) {
        if (!c || !launches) return;
        const bool on = c->profile == 2 || (c->profile == 3 && stage == H4D_STAGE_BLEND_FWD) ||
                        (c->profile == 4 && stage == H4D_STAGE_BLEND_BWD);
        if (!on) return;
        a = c->event();
        b = a ? c->event() : nullptr;
        if (!b && a) {
            c->pool.push_back(a);
            a = nullptr;
        }
    }
    ~KernelMark() {
        if (a && b) c->marks.push_back(h4d_ctx::Mark{a, b, stage});
    }
};

h4d_status hip_check(h4d_ctx* c, const char* where) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, H4D_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
    return H4D_OK;
}

constexpr size_t kAlign = 256;
constexpr size_t kPixelAlign = (size_t)1 << 21;
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
    int sx, sy, super_base;
    int64_t pix_base;
};

int bits_for(int n) {
    int b = 1;
    while ((1ll << b) < (long long)n) ++b;
    return b;
}

// LSD passes for a key of `bits` bits with digits of at most `width` bits, of
// near-equal width.  The depth sort uses 8-bit digits (its blocks are few and a
// wide digit's per-block cost dominates); the super-tile sort up to 11.
constexpr int kDepthDigitBits = 8;
constexpr int kDepthSortItems = 2;  // 512 keys per block: ~500 blocks for 250k Gaussians
int n_passes_for(int bits, int width) { return (bits + width - 1) / width; }
// Digit width of pass p (shift bits done) of the super-tile sort over `bits`
// bits: an even split, except that of two passes the first (over the low,
// evenly spread bits) takes two bits fewer than the second, so that its
// scatter writes runs of twice the length per digit.
int coarse_pass_bits(int bits, int p, int shift) {
    const int passes = n_passes_for(bits, kMaxRadixBits);
    if (passes == 2 && p == 0) return bits / 2 - 1;
    return (bits - shift + (passes - p) - 1) / (passes - p);
}
int coarse_max_bits(int bits) {
    int m = 0;
    for (int p = 0, shift = 0; shift < bits; ++p) {
        const int nb = coarse_pass_bits(bits, p, shift);
        m = std::max(m, nb);
        shift += nb;
    }
    return m;
}

// One pass of binning + blending covers the views [v0, v1): every view alone
// (views processed one after another), or as many of the call's views as the
// pass's super-tile ids allow (batched).  supers counts the pass's super-tiles
// including its static groups' grids.
struct Pass {
    int v0, v1, tiles, supers;
};

struct Layout {
    int N = 0, V = 0, total_tiles = 0, total_supers = 0;
    int n3 = 0, n4 = 0;
    int64_t total_pix = 0;
    uint64_t cap = 0;    // capacity in (Gaussian, tile) slots, S^2 per coarse entry
    uint64_t ccap = 0;   // coarse (Gaussian, super-tile) entries of the call: cap / S^2
    ViewGeom vg[kMaxViews];
    int n_pass = 0;
    Pass passes[kMaxViews];
    bool fits = true;    // every view's super-tiles fit one pass's key range
    // shared static binning (one pass holding every view): static groups of
    // views with the same camera, their leader views and grids
    bool shared = false;
    int n_groups = 0;
    ViewShare share[kMaxViews];
    // state
    // (the gradient records st_g2 come last: an inference render needs only
    // infer_bytes of the state)
    size_t st_status, st_pair_base, st_views, st_recs, st_ckeys, st_cvals, st_cranges, st_thist, st_T, st_nc, st_C,
        st_tcost, infer_bytes, st_g2, st_tids, state_bytes;
    // scratch, forward use
    size_t sc_dkeys, sc_dvals, sc_dkeys2, sc_dvals2, sc_cnt, sc_rect, sc_offsets, sc_partials, sc_eff, sc_ceff,
        sc_pkeys, sc_pvals, sc_pkeys2, sc_pvals2, sc_hist, sc_totals, sc_shape, sc_spans, sc_runs, sc_wcnt, sc_woff, sc_wpart,
        fwd_bytes;
    size_t hist_words = 0, totals_words = 0;  // 32-bit words of the radix histogram / digit totals
    // scratch, backward use
    size_t sc_border, sc_okeys, sc_ovals, sc_okeys2, sc_ovals2, sc_ohist, sc_ototals, ohist_words, bwd_bytes;
    size_t scratch_bytes;

    int n_passes() const { return n_pass; }
    Pass pass(int k) const { return passes[k]; }
    // depth-ordered entries of a pass and their segment layout
    SegLayout segs(const Pass& P) const {
        const int nv = P.v1 - P.v0;
        return shared ? SegLayout{nv, n4, n3} : SegLayout{nv, N, 0};
    }
    int64_t entries(const Pass& P) const {
        const int nv = P.v1 - P.v0;
        return shared ? (int64_t)nv * n4 + (int64_t)n_groups * n3 : (int64_t)nv * N;
    }
};

// Views with the same camera (pose, intrinsics, image size): a batched call
// that repeats a camera at several times bins the 3D Gaussians once per camera.
bool same_camera(const h4d_view& a, const h4d_view& b) {
    return std::memcmp(a.world_to_cam, b.world_to_cam, sizeof(a.world_to_cam)) == 0 && a.fx == b.fx &&
           a.fy == b.fy && a.cx == b.cx && a.cy == b.cy && a.width == b.width && a.height == b.height;
}

Layout make_layout(int N, int n3, const h4d_view* views, int V, const h4d_config* cfg) {
    Layout L;
    L.N = N;
    L.V = V;
    L.n3 = n3;
    L.n4 = N - n3;
    L.cap = (uint64_t)std::max<int64_t>(0, cfg->pair_capacity);
    int tb = 0, sb = 0;
    int64_t pb = 0;
    const int S = super_factor(cfg->tile);
    L.ccap = L.cap / (uint64_t)(S * S);
    for (int v = 0; v < V; ++v) {
        ViewGeom& g = L.vg[v];
        g.tiles_x = ceil_div(views[v].width, cfg->tile);
        g.tiles_y = ceil_div(views[v].height, cfg->tile);
        g.sx = ceil_div(g.tiles_x, S);
        g.sy = ceil_div(g.tiles_y, S);
        g.tile_base = tb;
        g.super_base = sb;
        g.pix_base = pb;
        tb += g.tiles_x * g.tiles_y;
        sb += g.sx * g.sy;
        pb += (int64_t)views[v].width * views[v].height;
        if (g.sx * g.sy > kMaxPassSupers) L.fits = false;
    }
    L.total_tiles = tb;
    L.total_pix = pb;
    // static groups: each view's first view with the same camera leads its group
    for (int v = 0; v < V; ++v) {
        int lead = v;
        for (int u = 0; u < v; ++u)
            if (same_camera(views[u], views[v])) {
                lead = u;
                break;
            }
        L.share[v].static_view = lead;
        L.share[v].static_next = -1;
        L.share[v].group_leader = -1;
    }
    int n_groups = 0, group_supers = 0;
    bool repeats = false;
    for (int v = 0; v < V; ++v) {
        if (L.share[v].static_view == v) {
            L.share[n_groups].group_leader = v;
            ++n_groups;
            group_supers += L.vg[v].sx * L.vg[v].sy;
        } else {
            repeats = true;
        }
    }
    L.shared = cfg->batched && repeats && n3 > 0 && L.fits && (int64_t)sb + group_supers <= kMaxPassSupers;
    if (L.shared) {
        L.n_groups = n_groups;
        int gs = sb;
        for (int g = 0; g < n_groups; ++g) {
            const int lead = L.share[g].group_leader;
            int prev = -1;
            for (int v = 0; v < V; ++v)
                if (L.share[v].static_view == lead) {
                    L.share[v].static_group = g;
                    L.share[v].static_super_base = gs;
                    if (prev >= 0) L.share[prev].static_next = v;
                    prev = v;
                }
            gs += L.vg[lead].sx * L.vg[lead].sy;
        }
        L.total_supers = gs;
        L.n_pass = 1;
        L.passes[0] = Pass{0, V, tb, gs};
    } else {
        for (int v = 0; v < V; ++v) {
            L.share[v].static_view = v;
            L.share[v].static_group = -1;
            L.share[v].static_super_base = L.vg[v].super_base;
            L.share[v].static_next = -1;
            L.share[v].group_leader = -1;
        }
        L.total_supers = sb;
        // views one after another, or batched passes of consecutive views whose
        // super-tiles fit the key range
        for (int v = 0; v < V;) {
            int e = v + 1, supers = L.vg[v].sx * L.vg[v].sy;
            while (cfg->batched && e < V && supers + L.vg[e].sx * L.vg[e].sy <= kMaxPassSupers)
                supers += L.vg[e].sx * L.vg[e].sy, ++e;
            const int tiles = (e < V ? L.vg[e].tile_base : tb) - L.vg[v].tile_base;
            L.passes[L.n_pass++] = Pass{v, e, tiles, supers};
            v = e;
        }
    }
    int max_views = 1;
    for (int k = 0; k < L.n_pass; ++k) max_views = std::max(max_views, L.passes[k].v1 - L.passes[k].v0);
    const size_t n = (size_t)N, V_ = (size_t)V;
    const size_t np = n * (size_t)max_views;  // depth-ordered entries of the largest pass (bound)
    Carve s;
    L.st_status = s.take(sizeof(Status));
    L.st_pair_base = s.take(8 * (V_ + 1));
    L.st_views = s.take(sizeof(ViewParams) * V_);
    L.st_recs = s.take(sizeof(Rec) * n * V_);
    L.st_ckeys = s.take(4 * (size_t)L.ccap);
    L.st_cvals = s.take(4 * (size_t)L.ccap);
    L.st_cranges = s.take(16 * (size_t)L.total_supers);
    L.st_thist = s.take(4 * (size_t)kCostBuckets * V_);  // one per pass (at most V); cleared with the ranges
    // the per-pixel arrays and everything after them start on a 2 MiB
    // boundary, so that their placement does not move with the pair capacity
    // (the adjoint's time varied with it by up to 2.5 %)
    s.off = (s.off + kPixelAlign - 1) / kPixelAlign * kPixelAlign;
    L.st_T = s.take(4 * (size_t)pb);
    L.st_nc = s.take(4 * (size_t)pb);
    L.st_C = s.take(12 * (size_t)pb);
    L.st_tcost = s.take(4 * (size_t)tb);
    L.infer_bytes = s.off;
    L.st_g2 = s.take(4 * (size_t)kG2Stride * n * V_);
    L.st_tids = s.take(4 * (size_t)kTileIds * (size_t)tb);
    L.state_bytes = s.off;
    Carve f;
    L.sc_dkeys = f.take(4 * np);
    L.sc_dvals = f.take(4 * np);
    L.sc_dkeys2 = f.take(4 * np);
    L.sc_dvals2 = f.take(4 * np);
    L.sc_cnt = f.take(4 * np);
    L.sc_rect = f.take(8 * np);
    L.sc_offsets = f.take(8 * (np + 1));
    L.sc_partials = f.take(8 * ((size_t)coarse_count_blocks((int)std::min<size_t>(np, 0x7FFFFFFF)) + 2));
    L.sc_eff = f.take(8);
    L.sc_ceff = f.take(8);
    L.sc_pkeys = f.take(4 * (size_t)L.ccap);
    L.sc_pvals = f.take(4 * (size_t)L.ccap);
    L.sc_pkeys2 = f.take(4 * (size_t)L.ccap);
    L.sc_pvals2 = f.take(4 * (size_t)L.ccap);
    // widest digit of any pass's super-tile sort (the width is not monotone in
    // the super-tile count: 2048 super-tiles take one 11-bit pass, 3300 two
    // 6-bit passes)
    int cbits = 1;
    for (int k = 0; k < L.n_passes(); ++k)
        cbits = std::max(cbits, coarse_max_bits(bits_for(L.pass(k).supers)));
    // the depth sort's segments: a pass's views (all Gaussians, or the 4D ones
    // when shared) and the static groups (3D ones)
    size_t dwords = radix_hist_words(n, max_views, kDepthDigitBits, kDepthSortItems);
    if (L.shared)
        dwords = std::max(radix_hist_words((uint64_t)L.n4, V, kDepthDigitBits, kDepthSortItems),
                          radix_hist_words((uint64_t)L.n3, L.n_groups, kDepthDigitBits, kDepthSortItems));
    L.hist_words = std::max(radix_hist_words(L.ccap, 1, cbits, kSortItems), dwords);
    L.totals_words = (size_t)kMaxRadix * (size_t)max_views;
    L.sc_hist = f.take(4 * L.hist_words);
    L.sc_totals = f.take(4 * L.totals_words);
    L.sc_shape = cfg->cull ? f.take(sizeof(CullShape) * np) : 0;
    L.sc_spans = cfg->cull ? f.take(4 * (size_t)kSpanRows * np) : 0;
    L.sc_runs = f.take(4 * ((size_t)L.ccap / 256 + 2));
    // tile lists written out on request (h4dgs_tile_lists): per-tile counts,
    // their offsets and the scan's partial sums
    L.sc_wcnt = f.take(4 * (size_t)tb);
    L.sc_woff = f.take(8 * ((size_t)tb + 1));
    L.sc_wpart = f.take(8 * ((size_t)scan_blocks(tb) + 2));
    L.fwd_bytes = f.off;
    Carve b;
    L.sc_border = b.take(4 * (size_t)tb);
    // the tile order's sort (used when a pass has many tiles)
    L.sc_okeys = b.take(4 * (size_t)tb);
    L.sc_ovals = b.take(4 * (size_t)tb);
    L.sc_okeys2 = b.take(4 * (size_t)tb);
    L.sc_ovals2 = b.take(4 * (size_t)tb);
    L.ohist_words = radix_hist_words((uint64_t)tb, 1, kMaxRadixBits, kSortItems);
    L.sc_ohist = b.take(4 * L.ohist_words);
    L.sc_ototals = b.take(4 * (size_t)kMaxRadix);
    L.bwd_bytes = b.off;
    L.scratch_bytes = std::max(L.fwd_bytes, L.bwd_bytes);
    return L;
}

// Every radix pass the forward will launch fits the layout's histogram and
// digit-total buffers (checked on the host before anything is enqueued; the
// launcher checks each pass again).
// Depth sorts of a pass: segments of equal length starting at `offset` in the
// key arrays (the pass's views; with shared static binning, the views' 4D
// Gaussians and the static groups' 3D Gaussians).
struct DepthJob {
    size_t offset;
    int n_seg;
    int len;
};
// Keys per thread of a depth-sort job: two (more, smaller blocks) for short
// key sets, which are latency-bound; kSortItems from 2^19 keys on, where the
// longer digit runs of 2048-key blocks coalesce the scatter (one view of 1M
// Gaussians: 0.121 -> 0.100 ms; 32 views of 1M batched: 0.89 -> 0.60 ms;
// 250k keys: 0.068 -> 0.083 ms with them).
int depth_items(const DepthJob& j) {
    return (uint64_t)j.len * (uint64_t)j.n_seg >= (1ull << 19) ? kSortItems : kDepthSortItems;
}
int depth_jobs(const Layout& L, const Pass& P, DepthJob* jobs) {
    const int nv = P.v1 - P.v0;
    int n = 0;
    if (!L.shared) {
        jobs[n++] = DepthJob{0, nv, L.N};
        return n;
    }
    if (L.n4 > 0) jobs[n++] = DepthJob{0, nv, L.n4};
    if (L.n3 > 0) jobs[n++] = DepthJob{(size_t)nv * L.n4, L.n_groups, L.n3};
    return n;
}

bool plan_fits(const Layout& L) {
    for (int k = 0; k < L.n_passes(); ++k) {
        const Pass P = L.pass(k);
        DepthJob jobs[2];
        const int nj = depth_jobs(L, P, jobs);
        const int passes = n_passes_for(32, kDepthDigitBits);
        for (int q = 0; q < nj; ++q)
            for (int p = 0, shift = 0; p < passes; ++p) {
                const int nb = (32 - shift + (passes - p) - 1) / (passes - p);
                if (!radix_pass_fits((uint64_t)jobs[q].len, jobs[q].n_seg, nb, depth_items(jobs[q]), L.hist_words,
                                     L.totals_words))
                    return false;
                shift += nb;
            }
        const int bits = bits_for(P.supers);
        const int cp = n_passes_for(bits, kMaxRadixBits);
        for (int p = 0, shift = 0; p < cp; ++p) {
            const int nb = coarse_pass_bits(bits, p, shift);
            if (!radix_pass_fits(L.ccap, 1, nb, kSortItems, L.hist_words, L.totals_words)) return false;
            shift += nb;
        }
    }
    return true;
}

// 64-bit words the forward's init clears from st_cranges on: the super-tile
// list ranges and the blending cost histograms behind them
size_t range_words(const Layout& L) {
    return (L.st_thist + 4 * (size_t)kCostBuckets * (size_t)L.V - L.st_cranges + 7) / 8;
}

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

h4d_status check_config(h4d_ctx* c, const h4d_config* cfg) {
    if (!cfg) return fail(c, H4D_ERR_INVALID_ARG, "config is null");
    if (!composite_supported(cfg->tile, cfg->chunk))
        return fail(c, H4D_ERR_INVALID_ARG, "tile must be 8, 16 or 32 and chunk 64, 128, 256 or 512 (got %d, %d)",
                    cfg->tile, cfg->chunk);
    if (cfg->pair_capacity < 0) return fail(c, H4D_ERR_INVALID_ARG, "pair_capacity < 0");
    if (cfg->pair_capacity > (int64_t)0xFFFFFFFFll * 4)
        return fail(c, H4D_ERR_INVALID_ARG, "pair_capacity too large");
    if (cfg->batched != 0 && cfg->batched != 1) return fail(c, H4D_ERR_INVALID_ARG, "batched must be 0 or 1");
    if (cfg->cull != 0 && cfg->cull != 1) return fail(c, H4D_ERR_INVALID_ARG, "cull must be 0 or 1");
    return H4D_OK;
}

// A pass indexes its (view, Gaussian) pairs with 32-bit integers.
h4d_status check_pass_size(h4d_ctx* c, const h4d_config* cfg, int64_t N, int n_views) {
    const int64_t per = cfg->batched ? n_views : 1;
    if (N * per > (int64_t)0x7FFFFFFF)
        return fail(c, H4D_ERR_INVALID_ARG, "batched pass too large: %lld Gaussians x %lld views >= 2^31",
                    (long long)N, (long long)per);
    return H4D_OK;
}

// Every view's super-tiles fit one binning pass's key range (16 bits): images
// up to 16384 pixels square at 16- and 32-pixel tiles, 8192 at 8-pixel tiles.
h4d_status check_layout(h4d_ctx* c, const Layout& L, const h4d_config* cfg) {
    if (L.fits) return H4D_OK;
    return fail(c, H4D_ERR_UNSUPPORTED, "a view has more than %d super-tiles of %d x %d pixels", kMaxPassSupers,
                cfg->tile * super_factor(cfg->tile), cfg->tile * super_factor(cfg->tile));
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
    if (g4->sh_t_degree < 0 || g4->sh_t_degree > kMaxTimeDeg)
        return fail(c, H4D_ERR_INVALID_ARG, "4D set: sh_t_degree %d not in [0, %d]", g4->sh_t_degree, kMaxTimeDeg);
    if (g4->sh_t_degree > 0 && (!(g4->sh_t_period > 0.f) || !std::isfinite(g4->sh_t_period) ||
                                (g4->n > 0 && !g4->sh_t)))
        return fail(c, H4D_ERR_INVALID_ARG, "4D set: time coefficients need sh_t and a finite period > 0");
    return H4D_OK;
}

// An output mirror of a 4D set with time coefficients must have room for them.
h4d_status check_time_out(h4d_ctx* c, const h4d_g4d* in4, const h4d_g4d_mut* out4, int32_t rows, const char* what) {
    if (in4->sh_t_degree > 0 && rows > 0 && !out4->sh_t)
        return fail(c, H4D_ERR_INVALID_ARG, "%s: the 4D set has time coefficients, the output has no sh_t", what);
    return H4D_OK;
}

G3Ptr to_ptr(const h4d_g3d* g) { return G3Ptr{g->n, g->mean, g->log_scale, g->quat, g->opacity, g->sh}; }
G4Ptr to_ptr(const h4d_g4d* g) {
    return G4Ptr{g->n,      g->mean,        g->mean_t,          g->log_scale, g->quat_l, g->quat_r,
                 g->opacity, g->sh, g->sh_t_degree, g->sh_t_period, g->sh_t};
}

ViewTableIn view_table(const h4d_view* views, int V, int tile, const Layout& L) {
    ViewTableIn t;
    std::memset(&t, 0, sizeof(t));
    t.n = V;
    t.tile = tile;
    for (int v = 0; v < V; ++v) t.share[v] = L.share[v];
    for (int v = 0; v < V; ++v) {
        ViewIn& o = t.v[v];
        std::memcpy(o.M, views[v].world_to_cam, sizeof(o.M));
        o.fx = views[v].fx; o.fy = views[v].fy; o.cx = views[v].cx; o.cy = views[v].cy;
        o.W = views[v].width; o.H = views[v].height; o.t = views[v].t;
        for (int k = 0; k < 3; ++k) o.bg[k] = views[v].bg[k];
    }
    return t;
}


unsigned long long* stat_counters(h4d_ctx* c, void* state, const Layout& L) {
    return c->stats ? reinterpret_cast<unsigned long long*>(&at<Status>(state, L.st_status)->pad[0]) : nullptr;
}

// The call's sorted coarse lists in its state.
CoarseLists coarse_lists(const Layout& L, const void* state) {
    void* s = const_cast<void*>(state);
    return CoarseLists{at<uint32_t>(s, L.st_ckeys), at<uint32_t>(s, L.st_cvals), at<int64_t>(s, L.st_cranges)};
}

// Binning and sorting of one pass whose records and depth keys are in place
// (Alg. 1 from DuplicateWithKeys to IdentifyTileRanges): its coarse lists go to
// the state's coarse arrays from cbase[P.v0] on, their ranges to st_cranges.
// Returns false (after launching only part of the pass) when a radix pass did
// not fit its buffers, which plan_fits rules out beforehand.
bool bin_pass(h4d_ctx* c, const Layout& L, const Pass& P, int tile, int cull, void* state, void* scratch,
              hipStream_t st, bool keep) {
    const int N = L.N;
    const int nv = P.v1 - P.v0;
    const int n = (int)L.entries(P);  // depth-ordered entries of the pass (segment layout)
    const SegLayout sg = L.segs(P);
    const Rec* recs = at<Rec>(state, L.st_recs);
    const ViewParams* vp = at<ViewParams>(state, L.st_views);
    uint32_t* dk = at<uint32_t>(scratch, L.sc_dkeys);
    uint32_t* dv = at<uint32_t>(scratch, L.sc_dvals);
    uint32_t* dk2 = at<uint32_t>(scratch, L.sc_dkeys2);
    uint32_t* dv2 = at<uint32_t>(scratch, L.sc_dvals2);
    uint32_t* hist = at<uint32_t>(scratch, L.sc_hist);
    uint32_t* totals = at<uint32_t>(scratch, L.sc_totals);
    {
        // depth order per segment: stable LSD passes over the float32 depth bits
        StageScope sc(c, st, H4D_STAGE_DEPTH_SORT);
        DepthJob jobs[2];
        const int nj = depth_jobs(L, P, jobs);
        const int passes = n_passes_for(32, kDepthDigitBits);
        int shift = 0;
        for (int pass = 0; pass < passes; ++pass) {
            const int nb = (32 - shift + (passes - pass) - 1) / (passes - pass);
            for (int q = 0; q < nj; ++q) {
                const size_t o = jobs[q].offset;
                if (!launch_radix_pass(dk + o, dv + o, dk2 + o, dv2 + o, nullptr, (uint64_t)jobs[q].len,
                                       (uint64_t)jobs[q].len, shift, nb, hist, L.hist_words, totals, L.totals_words,
                                       nullptr, st, jobs[q].n_seg, (uint64_t)jobs[q].len, nullptr, 0,
                                       depth_items(jobs[q])))
                    return false;
            }
            std::swap(dk, dk2);
            std::swap(dv, dv2);
            shift += nb;
        }
    }
    // dk / dv now hold the depth-ordered keys and ids
    if (unsigned long long* sc = keep ? stat_counters(c, state, L) : nullptr)
        launch_count_onscreen(recs, N, L.n4, vp, P.v0, nv, sc + 6, st);
    Status* status = at<Status>(state, L.st_status);
    unsigned long long* cbase = at<unsigned long long>(state, L.st_pair_base);
    const int S = super_factor(tile);
    StageScope sc(c, st, H4D_STAGE_BINNING);
    unsigned long long* eff_c = at<unsigned long long>(scratch, L.sc_eff);
    uint32_t* cnt = at<uint32_t>(scratch, L.sc_cnt);
    uint64_t* rect = at<uint64_t>(scratch, L.sc_rect);
    unsigned long long* offsets = at<unsigned long long>(scratch, L.sc_offsets);
    // coarse entries: one per (depth-ordered Gaussian, super-tile), the tile
    // mask in the key's upper half
    CullShape* shapes = cull ? at<CullShape>(scratch, L.sc_shape) : nullptr;
    uint32_t* spans = cull ? at<uint32_t>(scratch, L.sc_spans) : nullptr;
    unsigned long long* partials = at<unsigned long long>(scratch, L.sc_partials);
    launch_coarse_count(dv, n, N, sg, recs, vp, P.v0, tile, S, cnt, rect, shapes, spans, partials, st);
    uint32_t* runs = at<uint32_t>(scratch, L.sc_runs);
    launch_coarse_offsets(cnt, n, partials, L.ccap, S, cbase, P.v0, P.v1, status, eff_c, offsets, runs,
                          L.ccap / 256 + 1, st);
    uint32_t* pk = at<uint32_t>(scratch, L.sc_pkeys);
    uint32_t* pv = at<uint32_t>(scratch, L.sc_pvals);
    uint32_t* pk2 = at<uint32_t>(scratch, L.sc_pkeys2);
    uint32_t* pv2 = at<uint32_t>(scratch, L.sc_pvals2);
    launch_coarse_emit(offsets, runs, n, sg, rect, shapes, spans, vp, P.v0, tile, S, L.ccap, eff_c, pk, pv, st);
    // stable sort of the coarse entries by super-tile (depth order kept inside
    // each); the last pass writes the state's coarse arrays from cbase[P.v0]
    // on, with splat ids in place of the depth ranks.  The first pass also
    // drops the entries whose tile mask is empty (after culling, about 40 % of
    // them).  A single pass over the whole super-tile id also yields each
    // super-tile's list range; otherwise the ranges come from the sorted keys.
    const int bits = bits_for(P.supers);
    const int passes = n_passes_for(bits, kMaxRadixBits);
    int64_t* cranges = at<int64_t>(state, L.st_cranges) + 2 * (size_t)L.vg[P.v0].super_base;
    uint32_t* ckeys = at<uint32_t>(state, L.st_ckeys);
    uint32_t* cvals = at<uint32_t>(state, L.st_cvals);
    const unsigned long long* out0 = cbase + P.v0;
    uint32_t* kin = pk;
    uint32_t* vin = pv;
    int shift = 0;
    const bool drop = L.ccap > 0;  // (the first pass writes the kept count whenever it runs)
    unsigned long long* ceff = drop ? at<unsigned long long>(scratch, L.sc_ceff) : eff_c;  // entries kept
    for (int p = 0; p < passes; ++p) {
        const int nb = coarse_pass_bits(bits, p, shift);
        const bool last = p == passes - 1;
        uint32_t* kout = last ? ckeys : (kin == pk ? pk2 : pk);
        uint32_t* vout = last ? cvals : (vin == pv ? pv2 : pv);
        if (!launch_radix_pass(kin, vin, kout, vout, p == 0 ? eff_c : ceff, 0, L.ccap, shift, nb, hist,
                               L.hist_words, totals, L.totals_words, last ? out0 : nullptr, st, 1, 0,
                               passes == 1 ? cranges : nullptr, P.supers, kSortItems, last ? dv : nullptr,
                               (drop && p == 0) ? 1 : 0, (drop && p == 0) ? ceff : nullptr))
            return false;
        kin = kout;
        vin = vout;
        shift += nb;
    }
    if (passes > 1) {
        launch_fill_u64(reinterpret_cast<unsigned long long*>(cranges), 2 * (size_t)P.supers, 0ull, st);
        launch_ranges(ckeys, 0xFFFFu, ceff, out0, cranges, st);
    }
    return true;
}

// Every tile list of the call written out (ids: pair-capacity words; ranges:
// [start, end) per global tile).
void write_tile_lists(const Layout& L, int tile, void* state, void* scratch, uint32_t* ids, uint64_t ids_cap,
                      int64_t* ranges, hipStream_t st) {
    launch_walk_lists(tile, at<Rec>(state, L.st_recs), L.N, coarse_lists(L, state), L.shared,
                      at<ViewParams>(state, L.st_views), 0, L.V, L.total_tiles, at<uint32_t>(scratch, L.sc_wcnt),
                      at<unsigned long long>(scratch, L.sc_woff), at<unsigned long long>(scratch, L.sc_wpart), ids,
                      ids_cap, ranges, st);
}

// Blending of one pass whose coarse lists are in place.
// keep: write the adjoint's per-pixel and per-tile state (false for an
// inference render)
void blend_pass(h4d_ctx* c, const Layout& L, int k, int tile, int chunk, void* state, const PtrTable& images,
                hipStream_t st, bool keep) {
    const Pass P = L.pass(k);
    StageScope sc(c, st, H4D_STAGE_BLEND_FWD);
    KernelMark km(c, H4D_STAGE_BLEND_FWD, P.tiles > 0);
    launch_composite_fwd(tile, chunk, at<Rec>(state, L.st_recs), L.N, coarse_lists(L, state), L.shared,
                         at<ViewParams>(state, L.st_views), P.v0, P.v1, P.tiles, nullptr, images,
                         keep ? at<float>(state, L.st_T) : nullptr, keep ? at<uint32_t>(state, L.st_nc) : nullptr,
                         keep ? at<float>(state, L.st_C) : nullptr, keep ? at<uint32_t>(state, L.st_tcost) : nullptr,
                         keep ? at<uint32_t>(state, L.st_thist) + (size_t)kCostBuckets * k : nullptr,
                         keep ? at<uint32_t>(state, L.st_tids) : nullptr, keep ? stat_counters(c, state, L) : nullptr,
                         st, km.a, km.b);
}

constexpr int kNoallocDevices = 64;
std::mutex noalloc_mu;
char* noalloc_base[kNoallocDevices] = {};

// The current device's copy of noalloc_workspace, looked up on the first call
// on that device (with it current) and kept.
h4d_status noalloc_workspace_on_device(h4d_ctx* ctx, char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return hip_check(ctx, "render_infer_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kNoallocDevices)
        return fail(ctx, H4D_ERR_UNSUPPORTED, "render_infer_noalloc: device %d beyond %d", dev, kNoallocDevices);
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_base[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_workspace));
        if (e != hipSuccess || !p)
            return fail(ctx, H4D_ERR_HIP, "render_infer_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        noalloc_base[dev] = static_cast<char*>(p);
    }
    *out = noalloc_base[dev];
    return H4D_OK;
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
    if ((s = check_pass_size(ctx, cfg, (int64_t)n3 + n4, n_views)) != H4D_OK) return s;
    if (!state_bytes || !scratch_bytes) return fail(ctx, H4D_ERR_INVALID_ARG, "null size output");
    const Layout L = make_layout(n3 + n4, n3, views, n_views, cfg);
    if ((s = check_layout(ctx, L, cfg)) != H4D_OK) return s;
    *state_bytes = L.state_bytes;
    *scratch_bytes = L.scratch_bytes;
    return H4D_OK;
}

static h4d_status render_forward(h4d_ctx* ctx, const h4d_g3d* g3, const h4d_g4d* g4, const h4d_view* views,
                                 int32_t n_views, const h4d_config* cfg, float* const* images, void* state,
                                 size_t state_bytes, void* scratch, size_t scratch_bytes, void* stream, bool keep) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_sets(ctx, g3, g4)) != H4D_OK) return s;
    if ((s = check_config(ctx, cfg)) != H4D_OK) return s;
    if ((s = check_views(ctx, views, n_views)) != H4D_OK) return s;
    if ((s = check_pass_size(ctx, cfg, (int64_t)g3->n + g4->n, n_views)) != H4D_OK) return s;
    if (!images) return fail(ctx, H4D_ERR_INVALID_ARG, "images is null");
    for (int v = 0; v < n_views; ++v)
        if (!images[v]) return fail(ctx, H4D_ERR_INVALID_ARG, "image %d is null", v);
    const int N = g3->n + g4->n;
    const Layout L = make_layout(N, g3->n, views, n_views, cfg);
    if ((s = check_layout(ctx, L, cfg)) != H4D_OK) return s;
    const size_t need = keep ? L.state_bytes : L.infer_bytes;
    if (!state || state_bytes < need)
        return fail(ctx, H4D_ERR_INVALID_ARG, "state too small (%zu < %zu)", state_bytes, need);
    if (!scratch || scratch_bytes < L.fwd_bytes)
        return fail(ctx, H4D_ERR_INVALID_ARG, "scratch too small (%zu < %zu)", scratch_bytes, L.fwd_bytes);
    if (!plan_fits(L)) return fail(ctx, H4D_ERR_UNSUPPORTED, "internal: radix buffers of the layout too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const G3Ptr p3 = to_ptr(g3);
    const G4Ptr p4 = to_ptr(g4);
    ViewParams* vp = at<ViewParams>(state, L.st_views);
    launch_init_state(view_table(views, n_views, cfg->tile, L), vp, at<Status>(state, L.st_status),
                      at<unsigned long long>(state, L.st_pair_base), at<unsigned long long>(state, L.st_cranges),
                      range_words(L), st);
    PtrTable tab;
    std::memset(&tab, 0, sizeof(tab));
    for (int v = 0; v < n_views; ++v) tab.p[v] = images[v];
    for (int k = 0; k < L.n_passes(); ++k) {
        const Pass P = L.pass(k);
        {
            StageScope sc(ctx, st, H4D_STAGE_PREPROCESS);
            launch_preprocess(p3, p4, vp, P.v0, P.v1 - P.v0, L.shared ? 1 : 0, at<Rec>(state, L.st_recs),
                              at<uint32_t>(scratch, L.sc_dkeys), at<uint32_t>(scratch, L.sc_dvals),
                              keep ? at<float>(state, L.st_g2) : nullptr, st);
        }
        if (!bin_pass(ctx, L, P, cfg->tile, cfg->cull, state, scratch, st, keep))
            return fail(ctx, H4D_ERR_UNSUPPORTED, "internal: a radix pass did not fit its buffers");
        blend_pass(ctx, L, k, cfg->tile, cfg->chunk, state, tab, st, keep);
    }
    return hip_check(ctx, keep ? "render_fwd" : "render_infer");
}

h4d_status h4dgs_render_fwd(h4d_ctx* ctx, const h4d_g3d* g3, const h4d_g4d* g4, const h4d_view* views,
                            int32_t n_views, const h4d_config* cfg, float* const* images, void* state,
                            size_t state_bytes, void* scratch, size_t scratch_bytes, void* stream) {
    return render_forward(ctx, g3, g4, views, n_views, cfg, images, state, state_bytes, scratch, scratch_bytes,
                          stream, true);
}

h4d_status h4dgs_render_infer(h4d_ctx* ctx, const h4d_g3d* g3, const h4d_g4d* g4, const h4d_view* views,
                              int32_t n_views, const h4d_config* cfg, float* const* images, void* state,
                              size_t state_bytes, void* scratch, size_t scratch_bytes, void* stream) {
    return render_forward(ctx, g3, g4, views, n_views, cfg, images, state, state_bytes, scratch, scratch_bytes,
                          stream, false);
}

h4d_status h4dgs_render_infer_noalloc(h4d_ctx* ctx, const h4d_g3d* g3, const h4d_g4d* g4, const h4d_view* views,
                                      int32_t n_views, const h4d_config* cfg, float* const* images,
                                      uint64_t* status_out, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_sets(ctx, g3, g4)) != H4D_OK) return s;
    if ((s = check_config(ctx, cfg)) != H4D_OK) return s;
    if ((s = check_views(ctx, views, n_views)) != H4D_OK) return s;
    if ((s = check_pass_size(ctx, cfg, (int64_t)g3->n + g4->n, n_views)) != H4D_OK) return s;
    const Layout L = make_layout(g3->n + g4->n, g3->n, views, n_views, cfg);
    if ((s = check_layout(ctx, L, cfg)) != H4D_OK) return s;
    const size_t state_room = align_up(L.infer_bytes);
    const size_t limit = (size_t)H4DGS_NOALLOC_BYTES;
    if (state_room > limit || L.fwd_bytes > limit - state_room)
        return fail(ctx, H4D_ERR_CAPACITY,
                    "render_infer_noalloc: the call needs %zu bytes of workspace (state %zu + scratch %zu), "
                    "the fixed workspace holds %zu",
                    state_room + L.fwd_bytes, state_room, L.fwd_bytes, limit);
    char* base = nullptr;
    if ((s = noalloc_workspace_on_device(ctx, &base)) != H4D_OK) return s;
    if ((s = render_forward(ctx, g3, g4, views, n_views, cfg, images, base, state_room, base + state_room,
                            limit - state_room, stream, false)) != H4D_OK)
        return s;
    if (status_out) {
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (hipMemcpyAsync(status_out, base + L.st_status, 2 * sizeof(uint64_t), hipMemcpyDeviceToDevice, st) !=
            hipSuccess)
            return hip_check(ctx, "render_infer_noalloc: status copy");
    }
    return H4D_OK;
}

static h4d_status render_backward(h4d_ctx* ctx, const h4d_g3d* g3, const h4d_g4d* g4, const h4d_view* views,
                                  int32_t n_views, const h4d_config* cfg, const float* const* dl_dimages,
                                  void* state, size_t state_bytes, void* scratch, size_t scratch_bytes,
                                  h4d_g3d_mut* grad3, h4d_g4d_mut* grad4, const h4d_set_stats* stats3,
                                  const h4d_set_stats* stats4, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_sets(ctx, g3, g4)) != H4D_OK) return s;
    if ((s = check_config(ctx, cfg)) != H4D_OK) return s;
    if ((s = check_views(ctx, views, n_views)) != H4D_OK) return s;
    if ((s = check_pass_size(ctx, cfg, (int64_t)g3->n + g4->n, n_views)) != H4D_OK) return s;
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
    if ((s = check_time_out(ctx, g4, grad4, g4->n, "render_bwd")) != H4D_OK) return s;
    const int N = g3->n + g4->n;
    const Layout L = make_layout(N, g3->n, views, n_views, cfg);
    if ((s = check_layout(ctx, L, cfg)) != H4D_OK) return s;
    if (!state || state_bytes < L.state_bytes)
        return fail(ctx, H4D_ERR_INVALID_ARG, "state too small (%zu < %zu)", state_bytes, L.state_bytes);
    if (!scratch || scratch_bytes < L.bwd_bytes)
        return fail(ctx, H4D_ERR_INVALID_ARG, "scratch too small (%zu < %zu)", scratch_bytes, L.bwd_bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    void* stt = state;
    float* g2 = at<float>(stt, L.st_g2);
    Status* status = at<Status>(stt, L.st_status);
    uint32_t* border = at<uint32_t>(scratch, L.sc_border);
    // the forward zeroed the gradient records its on-screen pairs use; with
    // shared static binning the statistics need every view's own 3D records,
    // which it did not zero, and otherwise the 3D gradients of a static group
    // go to its view's records
    const bool want_stats = stats3 || stats4;
    const int static_rows = (L.shared && !want_stats) ? 1 : 0;
    PassTiles pt;
    pt.n = L.n_passes();
    for (int k = 0; k < pt.n; ++k) pt.tile0[k] = L.vg[L.pass(k).v0].tile_base;
    pt.tile0[pt.n] = L.total_tiles;
    const OrderSort osort{at<uint32_t>(scratch, L.sc_okeys),  at<uint32_t>(scratch, L.sc_ovals),
                          at<uint32_t>(scratch, L.sc_okeys2), at<uint32_t>(scratch, L.sc_ovals2),
                          at<uint32_t>(scratch, L.sc_ohist),  at<uint32_t>(scratch, L.sc_ototals),
                          L.ohist_words,                      (size_t)kMaxRadix};
    if (!launch_bwd_prologue(g2, (size_t)kG2Stride * N * n_views, &status->g2_dirty,
                             (L.shared && want_stats) ? 1 : 0, at<uint32_t>(stt, L.st_tcost),
                             at<uint32_t>(stt, L.st_thist), pt, osort, border, st))
        return fail(ctx, H4D_ERR_UNSUPPORTED, "internal: the tile order's sort did not fit its buffers");
    const ViewParams* vp = at<ViewParams>(stt, L.st_views);
    {
        StageScope sc(ctx, st, H4D_STAGE_BLEND_BWD);
        CPtrTable tab;
        std::memset(&tab, 0, sizeof(tab));
        for (int v = 0; v < n_views; ++v) tab.p[v] = dl_dimages[v];
        for (int k = 0; k < L.n_passes(); ++k) {
            const Pass P = L.pass(k);
            KernelMark km(ctx, H4D_STAGE_BLEND_BWD, P.tiles > 0);
            launch_composite_bwd(cfg->tile, cfg->chunk, at<Rec>(stt, L.st_recs), N, coarse_lists(L, stt),
                                 L.shared, static_rows, vp, P.v0, P.v1, P.tiles, border + pt.tile0[k], tab,
                                 at<float>(stt, L.st_T),
                                 at<uint32_t>(stt, L.st_nc), at<float>(stt, L.st_C), at<uint32_t>(stt, L.st_tids), g2,
                                 stat_counters(ctx, stt, L),
                                 st, km.a, km.b);
        }
    }
    const G3Grad r3{grad3->n, grad3->mean, grad3->log_scale, grad3->quat, grad3->opacity, grad3->sh};
    const G4Grad r4{grad4->n,       grad4->mean, grad4->mean_t, grad4->log_scale, grad4->quat_l, grad4->quat_r,
                    grad4->opacity, grad4->sh,   grad4->sh_t};
    const SetStats s3 = stats3 ? SetStats{stats3->grad_norm, stats3->visible, stats3->step_visible}
                               : SetStats{nullptr, nullptr, nullptr};
    const SetStats s4 = stats4 ? SetStats{stats4->grad_norm, stats4->visible, stats4->step_visible}
                               : SetStats{nullptr, nullptr, nullptr};
    {
        StageScope sc(ctx, st, H4D_STAGE_PREPROCESS_BWD);
        launch_preprocess_bwd(to_ptr(g3), to_ptr(g4), vp, n_views, at<Rec>(stt, L.st_recs), g2, r3, r4, s3, s4,
                              static_rows, status, st);
    }
    return hip_check(ctx, "render_bwd");
}

h4d_status h4dgs_render_bwd(h4d_ctx* ctx, const h4d_g3d* g3, const h4d_g4d* g4, const h4d_view* views,
                            int32_t n_views, const h4d_config* cfg, const float* const* dl_dimages, void* state,
                            size_t state_bytes, void* scratch, size_t scratch_bytes, h4d_g3d_mut* grad3,
                            h4d_g4d_mut* grad4, void* stream) {
    return render_backward(ctx, g3, g4, views, n_views, cfg, dl_dimages, state, state_bytes, scratch, scratch_bytes,
                           grad3, grad4, nullptr, nullptr, stream);
}

h4d_status h4dgs_render_bwd_stats(h4d_ctx* ctx, const h4d_g3d* g3, const h4d_g4d* g4, const h4d_view* views,
                                  int32_t n_views, const h4d_config* cfg, const float* const* dl_dimages,
                                  void* state, size_t state_bytes, void* scratch, size_t scratch_bytes,
                                  h4d_g3d_mut* grad3, h4d_g4d_mut* grad4, const h4d_set_stats* stats3,
                                  const h4d_set_stats* stats4, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    if (!stats3 || !stats4) return fail(ctx, H4D_ERR_INVALID_ARG, "null statistics descriptor");
    return render_backward(ctx, g3, g4, views, n_views, cfg, dl_dimages, state, state_bytes, scratch, scratch_bytes,
                           grad3, grad4, stats3, stats4, stream);
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
    const Layout L = make_layout(n, 0, &view, 1, cfg);
    if ((s = check_layout(ctx, L, cfg)) != H4D_OK) return s;
    if (!state || state_bytes < L.state_bytes) return fail(ctx, H4D_ERR_INVALID_ARG, "state too small");
    if (!scratch || scratch_bytes < L.fwd_bytes) return fail(ctx, H4D_ERR_INVALID_ARG, "scratch too small");
    if (!plan_fits(L)) return fail(ctx, H4D_ERR_UNSUPPORTED, "internal: radix buffers of the layout too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_init_state(view_table(&view, 1, cfg->tile, L), at<ViewParams>(state, L.st_views),
                      at<Status>(state, L.st_status), at<unsigned long long>(state, L.st_pair_base),
                      at<unsigned long long>(state, L.st_cranges), range_words(L), st);
    Rec* recs = at<Rec>(state, L.st_recs);
    launch_splats_to_records(n, u, v, conic, opacity, rgb, radius, depth, visible, width, height, recs,
                             at<uint32_t>(scratch, L.sc_dkeys), at<uint32_t>(scratch, L.sc_dvals), st);
    PtrTable tab;
    std::memset(&tab, 0, sizeof(tab));
    tab.p[0] = image;
    if (!bin_pass(ctx, L, L.pass(0), cfg->tile, cfg->cull, state, scratch, st, true))
        return fail(ctx, H4D_ERR_UNSUPPORTED, "internal: a radix pass did not fit its buffers");
    blend_pass(ctx, L, 0, cfg->tile, cfg->chunk, state, tab, st, true);
    const size_t hw = (size_t)width * height;
    if (T_final) (void)hipMemcpyAsync(T_final, at<float>(state, L.st_T), 4 * hw, hipMemcpyDeviceToDevice, st);
    if (sorted_ids && ranges)
        write_tile_lists(L, cfg->tile, state, scratch, sorted_ids, L.cap, ranges, st);
    return hip_check(ctx, "rasterize_splats");
}

h4d_status h4dgs_tile_lists(h4d_ctx* ctx, int32_t n3, int32_t n4, const h4d_view* views, int32_t n_views,
                            const h4d_config* cfg, const void* state, size_t state_bytes, void* scratch,
                            size_t scratch_bytes, uint32_t* ids, uint64_t ids_capacity, int64_t* ranges,
                            void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_config(ctx, cfg)) != H4D_OK) return s;
    if ((s = check_views(ctx, views, n_views)) != H4D_OK) return s;
    if (n3 < 0 || n4 < 0 || (int64_t)n3 + n4 > 0x7FFFFFFF) return fail(ctx, H4D_ERR_INVALID_ARG, "bad Gaussian counts");
    if ((s = check_pass_size(ctx, cfg, (int64_t)n3 + n4, n_views)) != H4D_OK) return s;
    const Layout L = make_layout(n3 + n4, n3, views, n_views, cfg);
    if ((s = check_layout(ctx, L, cfg)) != H4D_OK) return s;
    if (!state || state_bytes < L.state_bytes) return fail(ctx, H4D_ERR_INVALID_ARG, "state too small");
    if (!scratch || scratch_bytes < L.fwd_bytes) return fail(ctx, H4D_ERR_INVALID_ARG, "scratch too small");
    if (!ids || !ranges) return fail(ctx, H4D_ERR_INVALID_ARG, "ids / ranges is null");
    write_tile_lists(L, cfg->tile, const_cast<void*>(state), scratch, ids, ids_capacity, ranges,
                     static_cast<hipStream_t>(stream));
    return hip_check(ctx, "tile_lists");
}

h4d_status h4dgs_radix_pass_check(uint64_t capacity, int32_t n_seg, int32_t nbits, int32_t items,
                                  size_t hist_words, size_t totals_words) {
    return radix_pass_fits(capacity, n_seg, nbits, items, hist_words, totals_words) ? H4D_OK : H4D_ERR_INVALID_ARG;
}

size_t h4dgs_radix_hist_words(uint64_t capacity, int32_t n_seg, int32_t nbits, int32_t items) {
    return radix_hist_words(capacity, n_seg, nbits, items);
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
    if ((in3->n > 0 && (const void*)out3->mean == (const void*)in3->mean) ||
        (in4->n > 0 && (const void*)out4->mean == (const void*)in4->mean))
        return fail(ctx, H4D_ERR_INVALID_ARG, "outputs must not alias inputs");
    if ((s = check_time_out(ctx, in4, out4, in4->n, "convert_static")) != H4D_OK) return s;
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
    const G4Grad o4{out4->n,  out4->mean,    out4->mean_t, out4->log_scale, out4->quat_l, out4->quat_r,
                    out4->opacity, out4->sh, out4->sh_t};
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

size_t h4dgs_densify_scratch_bytes(int32_t n3, int32_t n4) {
    const size_t n = (size_t)std::max(0, std::max(n3, n4));
    const size_t nb = (size_t)std::max(1, scan_blocks((int)n));
    return align_up(3 * 4 * n) + align_up(3 * 8 * (n + 1)) + align_up(3 * 8 * (nb + 1)) + align_up(16);
}

namespace {
h4d_status check_densify_params(h4d_ctx* ctx, const h4d_densify_params* p, const char* which) {
    if (!p) return fail(ctx, H4D_ERR_INVALID_ARG, "%s: null densify parameters", which);
    if (p->split_n < 1 || p->split_n > 8) return fail(ctx, H4D_ERR_INVALID_ARG, "%s: split_n not in [1, 8]", which);
    if (!(p->grad_threshold >= 0.f) || !std::isfinite(p->grad_threshold))
        return fail(ctx, H4D_ERR_INVALID_ARG, "%s: grad_threshold must be finite and >= 0", which);
    if (std::isnan(p->log_dense_scale) || std::isnan(p->opacity_logit_min) || std::isnan(p->log_max_scale) ||
        !std::isfinite(p->log_shrink))
        return fail(ctx, H4D_ERR_INVALID_ARG, "%s: NaN limit or non-finite log_shrink", which);
    return H4D_OK;
}
DensifyP to_densify(const h4d_densify_params& p) {
    return DensifyP{p.grad_threshold, p.split_n, p.log_dense_scale, p.opacity_logit_min, p.log_max_scale,
                    p.log_shrink};
}
}  // namespace

h4d_status h4dgs_densify(h4d_ctx* ctx, const h4d_g3d* in3, const h4d_g4d* in4, const h4d_set_stats* st3,
                         const h4d_set_stats* st4, const float* noise3, const float* noise4,
                         const h4d_densify_params* p3, const h4d_densify_params* p4, h4d_g3d_mut* out3,
                         h4d_g4d_mut* out4, int32_t* src3, int32_t* src4, int32_t* n3_out, int32_t* n4_out,
                         void* scratch, size_t scratch_bytes, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_sets(ctx, in3, in4)) != H4D_OK) return s;
    if ((s = check_densify_params(ctx, p3, "3D")) != H4D_OK) return s;
    if ((s = check_densify_params(ctx, p4, "4D")) != H4D_OK) return s;
    if (!out3 || !out4 || !n3_out || !n4_out || !st3 || !st4) return fail(ctx, H4D_ERR_INVALID_ARG, "null output");
    const int64_t cap3 = (int64_t)in3->n * std::max(2, p3->split_n), cap4 = (int64_t)in4->n * std::max(2, p4->split_n);
    if (cap3 > 0x7FFFFFFF || cap4 > 0x7FFFFFFF) return fail(ctx, H4D_ERR_INVALID_ARG, "too many output rows");
    if (out3->n < cap3) return fail(ctx, H4D_ERR_CAPACITY, "out3 capacity %d < %lld", out3->n, (long long)cap3);
    if (out4->n < cap4) return fail(ctx, H4D_ERR_CAPACITY, "out4 capacity %d < %lld", out4->n, (long long)cap4);
    if (in3->n > 0 && (!st3->grad_norm || !st3->visible || !noise3 || !src3 || !out3->mean || !out3->log_scale ||
                       !out3->quat || !out3->opacity || !out3->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "3D set: null statistics, noise, src or output array");
    if (in4->n > 0 && (!st4->grad_norm || !st4->visible || !noise4 || !src4 || !out4->mean || !out4->mean_t ||
                       !out4->log_scale || !out4->quat_l || !out4->quat_r || !out4->opacity || !out4->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "4D set: null statistics, noise, src or output array");
    if ((in3->n > 0 && (const void*)out3->mean == (const void*)in3->mean) ||
        (in4->n > 0 && (const void*)out4->mean == (const void*)in4->mean))
        return fail(ctx, H4D_ERR_INVALID_ARG, "outputs must not alias inputs");
    if ((s = check_time_out(ctx, in4, out4, in4->n, "densify")) != H4D_OK) return s;
    const size_t need = h4dgs_densify_scratch_bytes(in3->n, in4->n);
    if (!scratch || scratch_bytes < need)
        return fail(ctx, H4D_ERR_INVALID_ARG, "scratch too small (%zu < %zu)", scratch_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)std::max(in3->n, in4->n);
    const size_t nb = (size_t)std::max(1, scan_blocks((int)n));
    Carve c;
    const size_t o_flags = c.take(3 * 4 * n), o_scan = c.take(3 * 8 * (n + 1)), o_part = c.take(3 * 8 * (nb + 1)),
                 o_cnt = c.take(16);
    int32_t* dcount = at<int32_t>(scratch, o_cnt);
    const G3Grad o3{out3->n, out3->mean, out3->log_scale, out3->quat, out3->opacity, out3->sh};
    const G4Grad o4{out4->n,  out4->mean,    out4->mean_t, out4->log_scale, out4->quat_l, out4->quat_r,
                    out4->opacity, out4->sh, out4->sh_t};
    int32_t hc[2] = {0, 0};
    // the sets one after another in the same scratch (each ends in a count read back)
    launch_densify3(to_ptr(in3), st3->grad_norm, st3->visible, noise3, to_densify(*p3), o3, src3,
                    at<uint32_t>(scratch, o_flags), at<unsigned long long>(scratch, o_scan),
                    at<unsigned long long>(scratch, o_part), dcount, st);
    if ((s = hip_check(ctx, "densify (3D)")) != H4D_OK) return s;
    if (hipMemcpyAsync(&hc[0], dcount, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return hip_check(ctx, "densify: count readback");
    launch_densify4(to_ptr(in4), st4->grad_norm, st4->visible, noise4, to_densify(*p4), o4, src4,
                    at<uint32_t>(scratch, o_flags), at<unsigned long long>(scratch, o_scan),
                    at<unsigned long long>(scratch, o_part), dcount, st);
    if ((s = hip_check(ctx, "densify (4D)")) != H4D_OK) return s;
    if (hipMemcpyAsync(&hc[1], dcount, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return hip_check(ctx, "densify: count readback");
    *n3_out = hc[0];
    *n4_out = hc[1];
    return H4D_OK;
}

h4d_status h4dgs_gather_rows(h4d_ctx* ctx, const h4d_g3d* in3, const h4d_g4d* in4, const int32_t* src3,
                             int32_t rows3, const int32_t* src4, int32_t rows4, h4d_g3d_mut* out3, h4d_g4d_mut* out4,
                             void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_sets(ctx, in3, in4)) != H4D_OK) return s;
    if (!out3 || !out4) return fail(ctx, H4D_ERR_INVALID_ARG, "null output");
    if (rows3 < 0 || rows4 < 0 || out3->n < rows3 || out4->n < rows4)
        return fail(ctx, H4D_ERR_INVALID_ARG, "row counts must be in [0, output capacity]");
    if (rows3 > 0 && (!src3 || !out3->mean || !out3->log_scale || !out3->quat || !out3->opacity || !out3->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "3D: null src or output array");
    if (rows4 > 0 && (!src4 || !out4->mean || !out4->mean_t || !out4->log_scale || !out4->quat_l || !out4->quat_r ||
                      !out4->opacity || !out4->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "4D: null src or output array");
    if ((s = check_time_out(ctx, in4, out4, rows4, "gather_rows")) != H4D_OK) return s;
    const G3Grad o3{out3->n, out3->mean, out3->log_scale, out3->quat, out3->opacity, out3->sh};
    const G4Grad o4{out4->n,  out4->mean,    out4->mean_t, out4->log_scale, out4->quat_l, out4->quat_r,
                    out4->opacity, out4->sh, out4->sh_t};
    launch_gather_rows(to_ptr(in3), src3, rows3, o3, to_ptr(in4), src4, rows4, o4, static_cast<hipStream_t>(stream));
    return hip_check(ctx, "gather_rows");
}

h4d_status h4dgs_convert_moments(h4d_ctx* ctx, const h4d_g4d* in4, const h4d_g3d* in3, const int32_t* perm,
                                 h4d_g4d_mut* out4, h4d_g3d_mut* out3, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_sets(ctx, in3, in4)) != H4D_OK) return s;
    if (!out4 || !out3) return fail(ctx, H4D_ERR_INVALID_ARG, "null output");
    if (out4->n < in4->n) return fail(ctx, H4D_ERR_CAPACITY, "out4 capacity %d < %d", out4->n, in4->n);
    if ((int64_t)out3->n < (int64_t)in3->n + in4->n)
        return fail(ctx, H4D_ERR_CAPACITY, "out3 capacity %d < %d", out3->n, in3->n + in4->n);
    if (in4->n > 0 && (!perm || !out4->mean || !out4->mean_t || !out4->log_scale || !out4->quat_l || !out4->quat_r ||
                       !out4->opacity || !out4->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "null 4D output array or perm");
    if (out3->n > 0 && (!out3->mean || !out3->log_scale || !out3->quat || !out3->opacity || !out3->sh))
        return fail(ctx, H4D_ERR_INVALID_ARG, "null 3D output array");
    if ((in3->n > 0 && (const void*)out3->mean == (const void*)in3->mean) ||
        (in4->n > 0 && (const void*)out4->mean == (const void*)in4->mean))
        return fail(ctx, H4D_ERR_INVALID_ARG, "outputs must not alias inputs");
    if ((s = check_time_out(ctx, in4, out4, in4->n, "convert_moments")) != H4D_OK) return s;
    const G4Grad o4{out4->n,  out4->mean,    out4->mean_t, out4->log_scale, out4->quat_l, out4->quat_r,
                    out4->opacity, out4->sh, out4->sh_t};
    const G3Grad o3{out3->n, out3->mean, out3->log_scale, out3->quat, out3->opacity, out3->sh};
    launch_convert_moments(to_ptr(in4), to_ptr(in3), perm, o4, o3, static_cast<hipStream_t>(stream));
    return hip_check(ctx, "convert_moments");
}

h4d_status h4dgs_adam(h4d_ctx* ctx, int32_t n_seg, float* const* params, const float* const* grads, float* const* m,
                      float* const* v, const int64_t* sizes, const float* lrs, double beta1, double beta2,
                      double eps, int32_t step, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    if (n_seg < 0 || n_seg > kMaxAdamSeg)
        return fail(ctx, H4D_ERR_INVALID_ARG, "n_seg must be in [0, %d]", kMaxAdamSeg);
    if (n_seg > 0 && (!params || !grads || !m || !v || !sizes || !lrs))
        return fail(ctx, H4D_ERR_INVALID_ARG, "null segment table");
    if (step < 1) return fail(ctx, H4D_ERR_INVALID_ARG, "step must be >= 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0))
        return fail(ctx, H4D_ERR_INVALID_ARG, "bad Adam constants");
    AdamTable t;
    std::memset(&t, 0, sizeof(t));
    t.n_seg = n_seg;
    t.b1 = (float)beta1; t.b2 = (float)beta2; t.eps = (float)eps;
    t.omb1 = (float)(1.0 - beta1);
    t.omb2 = (float)(1.0 - beta2);
    t.c1 = (float)(1.0 - std::pow(beta1, step));
    t.c2 = (float)(1.0 - std::pow(beta2, step));
    for (int i = 0; i < n_seg; ++i) {
        if (sizes[i] < 0) return fail(ctx, H4D_ERR_INVALID_ARG, "segment %d: negative size", i);
        if (sizes[i] > 0 && (!params[i] || !grads[i] || !m[i] || !v[i]))
            return fail(ctx, H4D_ERR_INVALID_ARG, "segment %d: null pointer", i);
        t.seg[i] = AdamSeg{params[i], grads[i], m[i], v[i], sizes[i], lrs[i], nullptr, 0};
    }
    {
        StageScope sc(ctx, static_cast<hipStream_t>(stream), H4D_STAGE_ADAM);
        launch_adam(t, static_cast<hipStream_t>(stream));
    }
    return hip_check(ctx, "adam");
}

h4d_status h4dgs_adam_masked(h4d_ctx* ctx, int32_t n_seg, float* const* params, const float* const* grads,
                             float* const* m, float* const* v, const int64_t* sizes, const float* lrs,
                             const uint8_t* const* masks, const int64_t* rows, double beta1, double beta2, double eps,
                             int32_t step, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    if (n_seg < 0 || n_seg > kMaxAdamSeg)
        return fail(ctx, H4D_ERR_INVALID_ARG, "n_seg must be in [0, %d]", kMaxAdamSeg);
    if (n_seg > 0 && (!params || !grads || !m || !v || !sizes || !lrs || !masks || !rows))
        return fail(ctx, H4D_ERR_INVALID_ARG, "null segment table");
    if (step < 1) return fail(ctx, H4D_ERR_INVALID_ARG, "step must be >= 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0))
        return fail(ctx, H4D_ERR_INVALID_ARG, "bad Adam constants");
    AdamTable t;
    std::memset(&t, 0, sizeof(t));
    t.n_seg = n_seg;
    t.b1 = (float)beta1; t.b2 = (float)beta2; t.eps = (float)eps;
    t.omb1 = (float)(1.0 - beta1);
    t.omb2 = (float)(1.0 - beta2);
    t.c1 = (float)(1.0 - std::pow(beta1, step));
    t.c2 = (float)(1.0 - std::pow(beta2, step));
    for (int i = 0; i < n_seg; ++i) {
        if (sizes[i] < 0) return fail(ctx, H4D_ERR_INVALID_ARG, "segment %d: negative size", i);
        if (sizes[i] > 0 && (!params[i] || !grads[i] || !m[i] || !v[i]))
            return fail(ctx, H4D_ERR_INVALID_ARG, "segment %d: null pointer", i);
        if (masks[i] && (rows[i] <= 0 || sizes[i] % rows[i] != 0))
            return fail(ctx, H4D_ERR_INVALID_ARG, "segment %d: size %lld is not a multiple of rows %lld", i,
                        (long long)sizes[i], (long long)rows[i]);
        t.seg[i] = AdamSeg{params[i], grads[i], m[i], v[i], sizes[i], lrs[i], masks[i], masks[i] ? rows[i] : 0};
    }
    {
        StageScope sc(ctx, static_cast<hipStream_t>(stream), H4D_STAGE_ADAM);
        launch_adam(t, static_cast<hipStream_t>(stream));
    }
    return hip_check(ctx, "adam_masked");
}

h4d_status h4dgs_l1_loss_grad(h4d_ctx* ctx, int32_t n_views, const float* const* images, const float* const* targets,
                              const h4d_view* views, float* const* dl_dimages, float* loss, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    h4d_status s;
    if ((s = check_views(ctx, views, n_views)) != H4D_OK) return s;
    if (!images || !targets || !dl_dimages) return fail(ctx, H4D_ERR_INVALID_ARG, "null image table");
    for (int v = 0; v < n_views; ++v) {
        if (!images[v] || !targets[v] || !dl_dimages[v]) return fail(ctx, H4D_ERR_INVALID_ARG, "null image %d", v);
        if (((uintptr_t)images[v] | (uintptr_t)targets[v] | (uintptr_t)dl_dimages[v]) % 16 != 0)
            return fail(ctx, H4D_ERR_INVALID_ARG, "image %d: buffers must be 16-byte aligned", v);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    StageScope sc(ctx, st, H4D_STAGE_LOSS);
    if (loss) launch_fill_f32(loss, 1, 0.f, st);  // a fill kernel: safe under graph capture
    for (int v = 0; v < n_views; ++v) {
        const size_t n = (size_t)3 * views[v].width * views[v].height;
        const float scale = (float)(1.0 / ((double)n * n_views));
        launch_l1_loss_grad(images[v], targets[v], dl_dimages[v], n, scale, loss, st);
    }
    return hip_check(ctx, "l1_loss_grad");
}

h4d_status h4dgs_profile(h4d_ctx* ctx, int32_t enable) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    if (enable < 0 || enable > 4) return fail(ctx, H4D_ERR_INVALID_ARG, "profile level %d not in [0, 4]", enable);
    ctx->profile = enable;
    return H4D_OK;
}

h4d_status h4dgs_profile_read(h4d_ctx* ctx, double* ms, int64_t* launches) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    if (!ms || !launches) return fail(ctx, H4D_ERR_INVALID_ARG, "null output");
    for (int k = 0; k < H4D_STAGE_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    h4d_status rc = H4D_OK;
    for (auto& m : ctx->marks) {
        float t = 0.f;
        if (hipEventSynchronize(m.b) != hipSuccess || hipEventElapsedTime(&t, m.a, m.b) != hipSuccess)
            rc = fail(ctx, H4D_ERR_HIP, "profile_read: event query failed");
        if (m.stage >= 0 && m.stage < H4D_STAGE_COUNT) {
            ms[m.stage] += t;
            launches[m.stage] += 1;
        }
        ctx->pool.push_back(m.a);
        ctx->pool.push_back(m.b);
    }
    ctx->marks.clear();
    return rc;
}

h4d_status h4dgs_stats(h4d_ctx* ctx, int32_t enable) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    ctx->stats = enable != 0;
    return H4D_OK;
}

h4d_status h4dgs_stats_read(h4d_ctx* ctx, const void* state, size_t state_bytes, int64_t* out, void* stream) {
    if (!ctx) return H4D_ERR_INVALID_ARG;
    if (!state || state_bytes < sizeof(Status) || !out) return fail(ctx, H4D_ERR_INVALID_ARG, "bad arguments");
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return hip_check(ctx, "stats_read");
    Status hs;
    if (hipMemcpy(&hs, state, sizeof(Status), hipMemcpyDeviceToHost) != hipSuccess) return hip_check(ctx, "stats_read");
    for (int k = 0; k < 7; ++k) out[k] = (int64_t)hs.pad[k];
    return H4D_OK;
}

}  // extern "C"

// Shared device-side definitions of the gfx950 rasterizer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace h4d {

// Rasterizer constants (the 3DGS-lineage constants the paper inherits by
// building on that implementation, Sec. 4.3).
constexpr double kNear = 0.2;
constexpr double kDilate = 0.3;
constexpr double kClampFov = 1.3;
constexpr double kEigFloor = 0.1;
constexpr double kSigmas = 3.0;
constexpr double kShOffset = 0.5;
constexpr float kMinAlpha = 1.0f / 255.0f;
constexpr double kMinAlphaD = 1.0 / 255.0;
constexpr float kMaxAlpha = 0.99f;
constexpr float kMinT = 1e-4f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr double kLn2 = 0.6931471805599453;  // 1 / log2(e)

constexpr int kMaxViews = 32;
constexpr uint32_t kCulledKey = 0xFFFFFFFFu;

// Per-view constants kept in device memory (written once per call).
struct ViewParams {
    double R[9];
    double T[3];
    double campos[3];  // camera centre in world coordinates, -R^T t
    double fx, fy, cx, cy, time;
    float bg[3];
    int32_t W, H;
    int32_t tiles_x, tiles_y;
    int32_t tile_base;   // first global tile id of this view
    int64_t pix_base;    // first pixel of this view in the concatenated pixel arrays
    int32_t sx, sy;      // super-tile grid (S x S tiles each)
    int32_t super_base;  // first global super-tile id of this view
    // Static binning shared by the views of one camera (a batched call whose
    // views repeat a camera at several times): the 3D Gaussians of this view
    // are projected, sorted and binned once, in the records of view
    // static_view, onto the super-tile grid of static group static_group, whose
    // first global super-tile id is static_super_base.  Unshared: static_view
    // is the view itself, static_group -1, static_super_base = super_base.
    int32_t static_view;
    int32_t static_group;
    int32_t static_super_base;
    int32_t static_next;  // the next view of the same static group (-1: none)
    // entry k of the table: the view whose records hold static group k (-1
    // past the last group)
    int32_t group_leader;
    int32_t pad;
};

// Tiles per super-tile edge: binning groups tiles into S x S blocks (S = 4 for
// 8- and 16-pixel tiles, 2 for 32-pixel tiles), so that a super-tile holds at
// most 16 tiles and a splat's tiles within it fit a 16-bit mask.
__host__ __device__ constexpr int super_factor(int tile) { return tile == 32 ? 2 : 4; }
// Super-tiles of one binning pass: their ids fill the low 16 bits of the coarse
// sort keys, the tile masks the high 16.
constexpr int kMaxPassSupers = 1 << 16;

// The view of global tile `gt` among views [v0, v1) (tile ids ascend with the view).
__device__ __forceinline__ int find_view_of_tile(const ViewParams* views, int v0, int v1, int gt) {
    int v = v0;
    while (v + 1 < v1 && views[v + 1].tile_base <= gt) ++v;
    return v;
}

// Sorted coarse lists of a call (binning's output, read by the blending
// kernels): per super-tile, its (Gaussian, super-tile) entries in depth order.
struct CoarseLists {
    const uint32_t* keys;   // super-tile id (pass-relative) | tile mask << 16
    const uint32_t* vals;   // splat id (relative to the record's view)
    const int64_t* ranges;  // [start, end) per global super-tile id
};

// Entries of each tile's list that the forward keeps (in walk order, with the
// static flag) for the adjoint, which re-walks only tiles whose last
// contributor lies beyond them.
constexpr int kTileIds = 256;

// Layout of a pass's depth-ordered entries: na segments of la entries (the
// views v0 .. v0 + na - 1, all their Gaussians, or only the 4D ones when the
// static binning is shared), then segments of lb entries, one per static group
// (the 3D Gaussians of the group's camera).
struct SegLayout {
    int na, la, lb;
};

// Screen-space gradients of one (view, Gaussian) from the blending adjoint:
// du dv dQ00 dQ01 dQ11 dop dr dg (conic entries unscaled, Q01 counted once;
// the first five summed without their constant factors and the effective
// opacity, which the projection adjoint applies) and db as four parts (slots 8-11, one per 16-lane row of the adjoint's
// reduction; their sum is db), padded to one 64-byte record so that a splat's
// atomic additions touch a single cache line.  Layout [view][N][kG2Stride].
// The forward zeroes the records of its on-screen (view, Gaussian) pairs; with
// shared static binning and no statistics wanted, the views of a static group
// add their 3D gradients into the records of the group's view.
constexpr int kG2Stride = 16;
constexpr int kG2Slots = 12;

// Per-view device pointers passed by value to the batched kernels.
struct PtrTable {
    float* p[kMaxViews];
};
struct CPtrTable {
    const float* p[kMaxViews];
};

// Screen-space record of one (Gaussian, view): 64 bytes, one half cache line.
//   a: (u - floor(u), v - floor(v), Q00', Q01')
//   b: (Q11', opacity, r, g)
//   c: (b, floor(u), floor(v), depth)         (floor values stored as float, exact)
//   d: (x0 | x1 << 16, y0 | y1 << 16, radius, 1 if covered else 0)
// Q' = Q * (-log2(e) / 2) with Q01' = Q01 * (-log2(e)), so that
// exp(power) = exp2(Q00' dx^2 + Q01' dx dy + Q11' dy^2).
struct __align__(16) Rec {
    float4 a, b, c;
    uint4 d;
};
static_assert(sizeof(Rec) == 64, "record is 64 bytes");

// Status words at the head of `state`.
struct Status {
    unsigned long long flags;        // bit 0: pair capacity overflow
    unsigned long long pairs_needed; // sum over views of the pairs the call needed
    // counters of the counting variants (h4dgs_stats): blend evaluations and
    // blends of the forward and the adjoint, tile-list entries, traversed
    // entries (each tile's last contributor) and on-screen records
    unsigned long long pad[13];
    // nonzero once a backward has accumulated into the screen-space gradient
    // records (which the forward leaves zeroed): a further backward clears them
    unsigned long long g2_dirty;
};

constexpr unsigned long long kFlagOverflow = 1ull;

// Parameter views (device pointers) as the kernels see them.
struct G3Ptr {
    int32_t n;
    const float *mean, *log_scale, *quat, *opacity, *sh;
};
struct G4Ptr {
    int32_t n;
    const float *mean, *mean_t, *log_scale, *quat_l, *quat_r, *opacity, *sh;
    // time coefficients of the colour: sh_t[48 sh_t_deg][n], terms cos(2 pi k
    // (t - mean_t) / sh_t_period), k = 1 .. sh_t_deg (0: plain SH)
    int32_t sh_t_deg;
    float sh_t_period;
    const float* sh_t;
};
struct G3Grad {
    int32_t n;
    float *mean, *log_scale, *quat, *opacity, *sh;
};
struct G4Grad {
    int32_t n;
    float *mean, *mean_t, *log_scale, *quat_l, *quat_r, *opacity, *sh;
    float* sh_t;  // [48 sh_t_deg][n] of the matching input set, when it has any
};
constexpr int kMaxTimeDeg = 2;

// Optional per-Gaussian statistics of one backward call (any pointer may be
// null): grad += sum over the views in which the Gaussian covers a pixel of
// |dL/d(centre)| in normalised device coordinates, vis += the number of those
// views, step_vis = 1 if there is one, else 0.
struct SetStats {
    float* grad;
    float* vis;
    uint8_t* step_vis;
};

// One view's share: the image-plane gradient (pixels) of the centre, scale
// times (e0, e1), in normalised device coordinates (half the image size per
// unit).
__device__ inline double ndc_grad_norm(float e0, float e1, double scale, int W, int H) {
    const double gx = (double)e0 * scale * (0.5 * (double)W), gy = (double)e1 * scale * (0.5 * (double)H);
    return sqrt(gx * gx + gy * gy);
}

__device__ inline void write_stats(const SetStats& st, int i, double gsum, int nvis) {
    if (st.grad) st.grad[i] += (float)gsum;
    if (st.vis) st.vis[i] += (float)nvis;
    if (st.step_vis) st.step_vis[i] = nvis > 0 ? 1 : 0;
}

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Dispatch-order bucket of a tile whose adjoint walks `cost` list entries:
// 0 for the most expensive (costs of 1023 and more share bucket 0).
constexpr int kCostBuckets = 1024;
__device__ __forceinline__ uint32_t cost_bucket(uint32_t cost) {
    return (uint32_t)(kCostBuckets - 1) - min(cost, (uint32_t)(kCostBuckets - 1));
}

// One front-to-back blending step, shared bit-for-bit by the forward and the
// backward kernels (the backward recomputes transmittance instead of storing it,
// so both must take every decision identically).  Inputs are the LDS copy of a
// record; dx, dy are pixel-centre minus splat-centre offsets.
struct Splat {
    float ui, vi, uf, vf;  // integer and fractional parts of the centre
    float qa, qb, qc;      // scaled conic (see Rec)
    float op;              // effective opacity
    float cr, cg, cb;
    int32_t x0, x1, y0, y1;
};

// The blending test of one (pixel, splat) pair, branch-free, shared bit-for-bit
// by the forward and backward kernels (the backward recomputes transmittance
// instead of storing it, so both must take every decision identically).  It is
// split into a column part, computed once for all pixels a lane holds in one
// column, and a per-pixel part.  power2 = log2(e) * power.

// Column part: pixel-centre x minus splat-centre x, its conic term and the
// x half of the square test.
// Column part of the quadratic form p2 = qa dx^2 + qb dx dy + qc dy^2 (shared
// by a lane's pixels): qa dx^2 and qb dx, so that each pixel adds
// dy (qc dy + qb dx) with two fused multiply-adds.
struct ColTerm {
    float dx, qadx, a2, bx;  // dx, qa dx, qa dx^2, qb dx
    bool inx;
};

__device__ __forceinline__ ColTerm eval_col(const Splat& s, int px, float pxc) {
#pragma clang fp contract(off)
    ColTerm c;
    c.inx = px >= s.x0 && px <= s.x1;
    c.dx = (pxc - s.ui) - s.uf;
    c.qadx = s.qa * c.dx;
    c.a2 = c.qadx * c.dx;
    c.bx = s.qb * c.dx;
    return c;
}

// Per-pixel part: returns whether the pair passes the square test (in: the
// pixel lies in the splat's pixel square), power <= 0 and alpha >= 1/255;
// alpha = min(0.99, op * exp(power)).
__device__ __forceinline__ bool eval_pix(const Splat& s, const ColTerm& c, bool in, float pyc, float& dy, float& G,
                                         float& alpha, bool& clamped) {
#pragma clang fp contract(off)
    dy = (pyc - s.vi) - s.vf;
    const float u = __builtin_fmaf(s.qc, dy, c.bx);
    const float p2 = __builtin_fmaf(dy, u, c.a2);
    G = __builtin_amdgcn_exp2f(p2);
    const float ap = s.op * G;
    clamped = ap > kMaxAlpha;
    alpha = __builtin_fminf(ap, kMaxAlpha);  // ap is never NaN
    return in && !(p2 > 0.0f) && alpha >= kMinAlpha;
}

// T (1 - alpha) as T - alpha T in one fused operation (exact T for alpha = 0).
__device__ __forceinline__ float next_T(float T, float alpha) { return __builtin_fmaf(-alpha, T, T); }

}  // namespace h4d

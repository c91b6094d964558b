// Host-side launchers of the gfx950 kernels (one translation unit per stage).
#pragma once

#include "common.hpp"

namespace h4d {

// Mirror of h4d_view (kept free of the public header so kernels see plain PODs).
struct ViewIn {
    float M[12];
    float fx, fy, cx, cy;
    int32_t W, H;
    float t;
    float bg[3];
};
// Per view: the shared static binning (ViewParams' static_* fields, filled by
// the host) and, at index k, the leader view of static group k (or -1).
struct ViewShare {
    int32_t static_view, static_group, static_super_base, static_next, group_leader;
};
struct ViewTableIn {
    int32_t n;
    int32_t tile;
    ViewIn v[kMaxViews];
    ViewShare share[kMaxViews];
};

// preprocess.hip
// The view table, cleared status / list-slot bases and empty tile ranges.
void launch_init_state(const ViewTableIn& in, ViewParams* views, Status* status, unsigned long long* pair_base,
                       unsigned long long* ranges, size_t n_range_words, hipStream_t st);
// Counting variant: the on-screen (view, Gaussian) records of views [v0, v0 +
// nv) (3D Gaussians read from each view's static_view), added to *counter.
void launch_count_onscreen(const Rec* recs, int N, int n4, const ViewParams* views, int v0, int nv,
                           unsigned long long* counter, hipStream_t st);
// Records of views [v0, v0 + nv) (recs: all views, [view][N]), depth keys and
// ids in the pass's segment layout: unshared (shared = 0), view v0 + r's at
// r * N; shared, view v0 + r's 4D Gaussians at r * n4 and the 3D Gaussians of
// static group g (computed for its leader view only) at nv * n4 + g * n3.
// g2 (may be null): zeroed for every record that covers a pixel.
void launch_preprocess(const G3Ptr& g3, const G4Ptr& g4, const ViewParams* views, int v0, int nv, int shared,
                       Rec* recs, uint32_t* dkeys, uint32_t* dvals, float* g2, hipStream_t st);
// static_rows: the adjoint added each static group's 3D gradients into the
// records of the group's view (no statistics then).  Marks g2 used
// (status->g2_dirty).
void launch_preprocess_bwd(const G3Ptr& g3, const G4Ptr& g4, const ViewParams* views, int n_views, const Rec* recs,
                           const float* g2, const G3Grad& gr3, const G4Grad& gr4, const SetStats& st3,
                           const SetStats& st4, int static_rows, Status* status, hipStream_t st);
void launch_splats_to_records(int n, const float* u, const float* v, const float* conic, const float* opacity,
                              const float* rgb, const int32_t* radius, const float* depth, const uint8_t* visible,
                              int W, int H, Rec* recs, uint32_t* dkeys, uint32_t* dvals, hipStream_t st);

// sort.hip
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kScanTile = 2048;

constexpr int kMaxRadixBits = 11;
constexpr int kMaxRadix = 1 << kMaxRadixBits;

// blocks of one pass over `capacity` keys with `items` keys per thread
int radix_blocks(uint64_t capacity, int items);
// words of `hist` for passes of up to max_bits bits
size_t radix_hist_words(uint64_t capacity, int n_seg, int max_bits, int items);
// Whether a pass fits histogram / digit-total buffers of the given sizes (in
// 32-bit words): hist needs radix_hist_words(capacity, n_seg, nbits, items),
// totals 2^nbits * n_seg; nbits in [1, 11], items kSortItems or 2 (8-bit
// digits only).
bool radix_pass_fits(uint64_t capacity, int n_seg, int nbits, int items, size_t hist_words, size_t totals_words);
// One stable LSD pass over `nbits` (<= 11) bits at `shift`, independently on
// n_seg segments that start seg_stride elements apart (all arrays).  Count
// (per segment) from *dcount when dcount != null, else hcount; capacity bounds
// the count.  Output positions (keys, values, digit ranges) are offset by
// *out_offset when out_offset != null.
// hist / totals hold hist_words / totals_words words; a pass that does not fit
// them (radix_pass_fits) launches nothing and returns false.  items: keys per
// thread, kSortItems or 2 (8-bit digits only; for short key sets, more and
// smaller blocks).
// digit_ranges (may be null): for a pass over whole keys, [start, end) of each
// of the first n_digit_ranges digits in the output.  val_map (may be null):
// the values written out are val_map[value].  skip_empty: keys whose upper 16
// bits are zero are dropped (the output holds the others, in order, from
// position 0); out_count (may be null) receives the number of keys written.
bool launch_radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
                       const unsigned long long* dcount, uint64_t hcount, uint64_t capacity, int shift, int nbits,
                       uint32_t* hist, size_t hist_words, uint32_t* totals, size_t totals_words,
                       const unsigned long long* out_offset, hipStream_t st, int n_seg = 1, uint64_t seg_stride = 0,
                       int64_t* digit_ranges = nullptr, int n_digit_ranges = 0, int items = kSortItems,
                       const uint32_t* val_map = nullptr, int skip_empty = 0,
                       unsigned long long* out_count = nullptr);
int scan_blocks(int n);
// out[j] = sum_{i<j} in[idx[i]] (idx may be null), out[n] = total; 64-bit.
// With run_start, run_start[r] (r < run_cap) receives the index i whose range
// [out[i], out[i + 1]) holds output 256 r.
void launch_scan_u32_u64(const uint32_t* in, const uint32_t* idx, int n, unsigned long long* out,
                         unsigned long long* partials, hipStream_t st, uint32_t* run_start = nullptr,
                         uint64_t run_cap = 0);
// The alpha >= 1/255 region of one splat as the binning's tile test needs it:
// -p2 = a dx^2 - b dx dy + c dy^2 <= t, with dx, dy offsets from the centre (set
// up in FP64 per splat, tested in FP32 on widened intervals).
struct __align__(16) CullShape {
    float b, inv2a, four_at, det4;  // det4 = 4ac - b^2
    float y_full, y_ext;            // half-height; height of the rightmost point
    float pad_x, pad_y;
    float ui, uf, vi, vf;           // centre, integer and fractional parts
    int px0, px1, py0, py1;         // pixel square
    int mode;                       // 0: keep every tile, 1: test, 2: no pixel can pass
};
// Tile rows whose column spans the count kernel tabulates per splat (taller
// splats keep their CullShape and are tested per coarse entry).
constexpr int kSpanRows = 16;

// Two-level binning over the views [v0, v1) of one pass; j indexes the pass's
// depth-ordered entries in the segment layout sg (n entries; sorted_gid[j]:
// the splat id, relative to its record's view).  Super-tile ids are relative to
// view v0's first (a pass holds at most kMaxPassSupers of them).
// partials: coarse_count_blocks(n) + 1 words, each count workgroup's sum.
// Culling (shapes and spans non-null, n CullShapes and kSpanRows n words): the
// tile rectangle shrinks to the tiles the alpha >= 1/255 test can keep, and the
// test's per-row column spans are tabulated (or, for taller splats, the shape
// kept) for the emission.
int coarse_count_blocks(int n);
void launch_coarse_count(const uint32_t* sorted_gid, int n, int N, SegLayout sg, const Rec* recs,
                         const ViewParams* views, int v0, int tile, int S, uint32_t* cnt, uint64_t* rect_sorted,
                         CullShape* shapes, uint32_t* spans, unsigned long long* partials, hipStream_t st);
// offsets[j] = sum of cnt before j (offsets[n] = C) with run_start as in
// launch_scan_u32_u64; capacity check: the pass's C coarse entries go to
// [cbase[v0], cbase[v0] + C) of the call's ccap; cbase[v1] receives the end
// and status->pairs_needed grows by S^2 C; *eff_count = C, or 0 on overflow.
void launch_coarse_offsets(const uint32_t* cnt, int n, unsigned long long* partials, uint64_t ccap, int S,
                           unsigned long long* cbase, int v0, int v1, Status* status, unsigned long long* eff_count,
                           unsigned long long* offsets, uint32_t* run_start, uint64_t run_cap, hipStream_t st);
// Keys carry each entry's tile mask in their upper 16 bits (cull: less the
// tiles no pixel of which can reach alpha >= 1/255).
void launch_coarse_emit(const unsigned long long* offsets, const uint32_t* run_start, int n, SegLayout sg,
                        const uint64_t* rect_sorted, const CullShape* shapes, const uint32_t* spans,
                        const ViewParams* views, int v0, int tile, int S, uint64_t capacity,
                        const unsigned long long* eff_count, uint32_t* keys, uint32_t* vals, hipStream_t st);
// ranges of the sorted keys keys[*base ..) (compared under key_mask):
// ranges[2k], ranges[2k+1] = [first, last+1), counted from keys (base may be
// null: 0)
void launch_ranges(const uint32_t* keys, uint32_t key_mask, const unsigned long long* eff_count,
                   const unsigned long long* base, int64_t* ranges, hipStream_t st);
// Backward prologue: zeroes g2[0, n_g2) if *dirty != 0 or force, and orders the
// tiles of every pass by decreasing tcost: one workgroup per pass from the
// forward's bucket counts, or, when a pass has more than kOrderBlockTiles
// tiles, by a radix sort over the buffers of `sort` (keys, vals, keys2, vals2:
// one word per tile; hist / totals as the radix pass needs for that many keys
// and 11-bit digits).  Returns false if a sort pass did not fit its buffers. (pass k: global tiles [tile0[k], tile0[k + 1]), its order
// at the same offsets, relative to tile0[k]; thist + k kCostBuckets: the
// forward's per-bucket tile counts of pass k).  A permutation whatever the
// counts hold: buckets that overflow fall back to identity order.
struct PassTiles {
    int32_t n;                     // passes
    int32_t tile0[kMaxViews + 1];
};
constexpr int kOrderBlockTiles = 32768;
struct OrderSort {
    uint32_t *keys, *vals, *keys2, *vals2, *hist, *totals;
    size_t hist_words, totals_words;
};
bool launch_bwd_prologue(float* g2, size_t n_g2, const unsigned long long* dirty, int force, const uint32_t* tcost,
                         const uint32_t* thist, const PassTiles& passes, const OrderSort& sort, uint32_t* order,
                         hipStream_t st);
void launch_fill_u64(unsigned long long* p, size_t n, unsigned long long val, hipStream_t st);
void launch_fill_f32(float* p, size_t n, float val, hipStream_t st);

// composite.hip
bool composite_supported(int tile, int chunk);
// One launch over the tiles of views [v0, v1) (n_tiles = their total): recs
// holds every view's records ([view][N]), lists the call's sorted coarse lists
// (merge: each tile merges its static group's 3D list with its own 4D list),
// images/dls are indexed by view and g2 holds kG2Stride floats per (view,
// Gaussian).  order (may be null: tile
// b = workgroup b): the n_tiles tiles (relative to the launch's first) in
// dispatch order, a permutation.  The forward writes, per tile, its last
// contributor into tcost[global tile] and counts the launch's tiles per
// cost_bucket into thist[kCostBuckets] (zero on entry) and keeps the first
// kTileIds entries of each tile's list in tids[global tile][kTileIds] (may be
// null), which the adjoint reads for tiles whose contributors all lie there.
// Non-null e0 / e1 receive the kernel's own start / end time.
void launch_composite_fwd(int tile, int chunk, const Rec* recs, int N, const CoarseLists& lists, bool merge,
                          const ViewParams* views, int v0, int v1, int n_tiles, const uint32_t* order,
                          const PtrTable& images, float* Tfin, uint32_t* ncontrib, float* Cout, uint32_t* tcost,
                          uint32_t* thist, uint32_t* tids, unsigned long long* counters, hipStream_t st,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// static_rows (merge only): the 3D entries' gradients go to the records of
// their static group's view instead of the tile's own view.
void launch_composite_bwd(int tile, int chunk, const Rec* recs, int N, const CoarseLists& lists, bool merge,
                          int static_rows, const ViewParams* views, int v0, int v1, int n_tiles,
                          const uint32_t* order, const CPtrTable& dls, const float* Tfin, const uint32_t* ncontrib,
                          const float* Cout, const uint32_t* tids, float* g2, unsigned long long* counters,
                          hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// The tile lists of the views [v0, v1) written out: ids (indices into the
// merged set [4D | 3D]) of tile t (relative to view v0's first tile) at
// out[offsets[t] ..) (positions from out_cap on are not written),
// ranges[global tile] = [offsets[t], offsets[t + 1]); cnt holds n_tiles
// words, offsets n_tiles + 1, partials scan_blocks(n_tiles) + 1.
void launch_walk_lists(int tile, const Rec* recs, int N, const CoarseLists& lists, bool merge,
                       const ViewParams* views, int v0, int v1, int n_tiles, uint32_t* cnt,
                       unsigned long long* offsets, unsigned long long* partials, uint32_t* out, uint64_t out_cap,
                       int64_t* ranges, hipStream_t st);
// L1 loss gradient (loss.hip)
void launch_l1_loss_grad(const float* img, const float* target, float* dl, size_t n, float scale, float* loss,
                         hipStream_t st);

// convert.hip
// Densification limits as the kernels take them (see h4d_densify_params).
struct DensifyP {
    float thr;
    int split_n;
    double log_dense, logit_min, log_max_scale, log_shrink;
};
void launch_densify3(const G3Ptr& g, const float* grad, const float* vis, const float* noise, const DensifyP& p,
                     const G3Grad& o, int32_t* src, uint32_t* flags, unsigned long long* scan,
                     unsigned long long* partials, int32_t* count, hipStream_t st);
void launch_densify4(const G4Ptr& g, const float* grad, const float* vis, const float* noise, const DensifyP& p,
                     const G4Grad& o, int32_t* src, uint32_t* flags, unsigned long long* scan,
                     unsigned long long* partials, int32_t* count, hipStream_t st);
void launch_gather_rows(const G3Ptr& g3, const int32_t* src3, int rows3, const G3Grad& o3, const G4Ptr& g4,
                        const int32_t* src4, int rows4, const G4Grad& o4, hipStream_t st);
void launch_convert_moments(const G4Ptr& in4, const G3Ptr& in3, const int32_t* perm, const G4Grad& out4,
                            const G3Grad& out3, hipStream_t st);
void launch_convert_static(const G4Ptr& in4, const G3Ptr& in3, double log_tau, const G4Grad& out4,
                           const G3Grad& out3, int32_t* perm, uint32_t* flags, unsigned long long* scan,
                           unsigned long long* partials, int32_t* counts, hipStream_t st);

// adam.hip
struct AdamSeg {
    float* p;
    const float* g;
    float* m;
    float* v;
    int64_t n;
    float lr;
    // optional row mask: element e belongs to row e % rows and is updated only
    // where mask[row] != 0 (parameter, moments unchanged elsewhere)
    const uint8_t* mask;
    int64_t rows;
};
constexpr int kMaxAdamSeg = 16;
struct AdamTable {
    int32_t n_seg;
    float b1, b2, omb1, omb2, eps, c1, c2;  // omb = 1 - b, c1 = 1 - b1^t, c2 = 1 - b2^t
    AdamSeg seg[kMaxAdamSeg];
};
void launch_adam(const AdamTable& t, hipStream_t st);

}  // namespace h4d

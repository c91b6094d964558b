// Front-to-back blending on gfx950 (Eq. 3; Alg. 1 BlendInOrder) and its adjoint.
//
// One workgroup per B x B tile (B = 8: one wave64; 16: one wave in the adjoint,
// two in the forward; 32: four waves), one to four pixels per lane, all of a
// lane's pixels in one column.  The tile's
// depth-ordered list is walked in chunks: the first wave pulls the chunk's
// entries from the sorted coarse lists (TileWalk), then each chunk of records
// is gathered once from HBM into LDS and broadcast to every lane.  A pixel's
// contributors are exactly the splats whose pixel square contains it, so the
// image does not depend on B or on the chunk size.
//
// The backward recomputes transmittance front to back with the very same
// blending test as the forward (eval_col / eval_pix, next_T).  The colour behind
// a splat enters dL/dalpha only through its dot product with dL/dC, kept per
// pixel as R = dot(dL/dC, C_out), less each blended splat's share in turn.  Each lane sums
// its pixels in registers; the nine per-splat gradients are reduced across the
// wave by reduce-scatter (lane-half and row swaps, DPP mirrors, quad sums; skipped
// when no lane blended the splat) and added to HBM with one global atomic
// instruction per (splat, wave), a lane per record slot.  Constant factors of the conic and centre
// gradients, and the splat's opacity, are applied where the record is read.  Each wave stops
// at its own last contributor.
#include <hip/hip_ext.h>
#include <type_traits>
#include "common.hpp"
#include "launch.hpp"
#include "walk.hpp"

namespace h4d {

// LDS copy of one record (64 bytes, 16-byte aligned so that a lane reads it
// with four 128-bit LDS loads): packed pixel square, centre split into integer
// and fractional parts, scaled conic, opacity, colour.  Bit 31 of ry (image
// rows stay below 2^15) is set when the square holds every pixel row of the
// tile: the blending loops then skip the per-pixel row test, and y0, y1 are
// not read.
struct __align__(16) LSplat {
    uint32_t rx, ry;              // x0 | x1 << 16, y0 | y1 << 16 (| rows-in flag << 31)
    float ui, uf, vi, vf;
    float qa, qb, qc, op;
    float cr, cg, cb;
    uint32_t gid;                 // splat id (used by the backward)
    float qa2, qc2;               // 2 qa, 2 qc (used by the backward)
};
static_assert(sizeof(LSplat) == 64, "LDS splat is 64 bytes");
constexpr uint32_t kRowsIn = 0x80000000u;

// row0, row1: the tile's first and last pixel rows
__device__ __forceinline__ void stage_splat(const Rec& r, uint32_t gid, int row0, int row1, LSplat& s) {
    s.gid = gid;
    s.rx = r.d.x;
    const uint32_t y0 = r.d.y & 0xFFFFu, y1 = r.d.y >> 16;
    s.ry = r.d.y | ((y0 <= (uint32_t)row0 && y1 >= (uint32_t)row1) ? kRowsIn : 0u);
    s.ui = r.c.y; s.uf = r.a.x; s.vi = r.c.z; s.vf = r.a.y;
    // qc < 0 for every conic (the dilated covariance is positive definite);
    // the bound keeps it below zero where a vast splat's value would round to
    // -0, so that a finished pixel's infinite row offset still gives power -inf
    s.qa = r.a.z; s.qb = r.a.w; s.qc = __builtin_fminf(r.b.x, -1.17549435e-38f); s.op = r.b.y;
    s.cr = r.b.z; s.cg = r.b.w; s.cb = r.c.x;
    s.qa2 = 2.0f * r.a.z; s.qc2 = 2.0f * s.qc;
}

// (y0, y1 as stored: only meaningful when the rows-in flag is clear)
__device__ __forceinline__ Splat to_splat(const LSplat& l) {
    Splat s;
    s.x0 = (int)(l.rx & 0xFFFFu); s.x1 = (int)(l.rx >> 16); s.y0 = (int)(l.ry & 0xFFFFu); s.y1 = (int)(l.ry >> 16);
    s.ui = l.ui; s.uf = l.uf; s.vi = l.vi; s.vf = l.vf;
    s.qa = l.qa; s.qb = l.qb; s.qc = l.qc; s.op = l.op;
    s.cr = l.cr; s.cg = l.cg; s.cb = l.cb;
    return s;
}

// The same record read as four 128-bit LDS loads from one address, with the
// adjoint's extra fields (2 qa, 2 qc).
__device__ __forceinline__ Splat to_splat_wide(const LSplat& l, float& qa2, float& qc2) {
    const uint4* p = reinterpret_cast<const uint4*>(&l);
    const uint4 w0 = p[0], w1 = p[1], w2 = p[2], w3 = p[3];
    Splat s;
    s.x0 = (int)(w0.x & 0xFFFFu); s.x1 = (int)(w0.x >> 16); s.y0 = (int)(w0.y & 0xFFFFu); s.y1 = (int)(w0.y >> 16);
    s.ui = __uint_as_float(w0.z); s.uf = __uint_as_float(w0.w);
    s.vi = __uint_as_float(w1.x); s.vf = __uint_as_float(w1.y);
    s.qa = __uint_as_float(w1.z); s.qb = __uint_as_float(w1.w);
    s.qc = __uint_as_float(w2.x); s.op = __uint_as_float(w2.y);
    s.cr = __uint_as_float(w2.z); s.cg = __uint_as_float(w2.w); s.cb = __uint_as_float(w3.x);
    qa2 = __uint_as_float(w3.z); qc2 = __uint_as_float(w3.w);
    return s;
}

// Rows-in flags of the staged splats [g0, g0 + n), n <= 64, as a wave-uniform
// bit mask (bit i: splat g0 + i).
__device__ __forceinline__ unsigned long long rows_in_mask(const LSplat* sp, int g0, int n) {
    const int lane = __lane_id();
    return __ballot(lane < n && (sp[g0 + lane].ry & kRowsIn) != 0u);
}

// First position at or after j whose bit in m is set, or n (n <= 64).
__device__ __forceinline__ int next_set(unsigned long long m, int j, int n) {
    if (j >= n) return n;
    const unsigned long long r = m >> j;
    return r ? min(n, j + (int)__builtin_ctzll(r)) : n;
}

// Calls step(j, tag) for j = 0 .. n-1 in order, tag = std::true_type where bit j
// of rin is set, else std::false_type; stops early (returning true) when step
// returns true.  Runs of equal flags go through their own counted loop (the
// run's end found once, from the mask), so that the loop-carried pixel state
// stays in place across each run and a step pays no mask test.
template <class F>
__device__ __forceinline__ bool walk_runs(unsigned long long rin, int n, F&& step) {
    int j = 0;
    while (j < n) {
        for (const int e = next_set(~rin, j, n); j < e; ++j)
            if (step(j, std::true_type{})) return true;
        for (const int e = next_set(rin, j, n); j < e; ++j)
            if (step(j, std::false_type{})) return true;
    }
    return false;
}

// Splats whose opacity lies below this never reach the 0.99 clamp: every pair
// that passes the power test has G = exp2(power) <= 1 (up to the exp2
// rounding, which the margin covers), so alpha = opacity * G < 0.99.
constexpr float kClampOp = 0.98f;

// Opacity flags of the staged splats [g0, g0 + n) (bit i: splat g0 + i may
// reach the clamp).
__device__ __forceinline__ unsigned long long clamp_mask(const LSplat* sp, int g0, int n) {
    const int lane = __lane_id();
    return __builtin_amdgcn_ballot_w64(lane < n && sp[g0 + lane].op >= kClampOp);
}

// The adjoint's walk: calls step(j, tag) for j = j0 .. n-1 in order, tag =
// std::integral_constant<int, f | X> with bit 0 of f set where bit j of rin is,
// bit 1 where bit j of clp is; each run of equal flags goes through its own
// counted loop.
template <int X, class F>
__device__ __forceinline__ void walk_runs2(unsigned long long rin, unsigned long long clp, int j0, int n, F&& step) {
    int j = j0;
    while (j < n) {
        for (const int e = next_set(~rin | clp, j, n); j < e; ++j) step(j, std::integral_constant<int, 1 | X>{});
        for (const int e = next_set(rin | clp, j, n); j < e; ++j) step(j, std::integral_constant<int, 0 | X>{});
        for (const int e = next_set(~rin | ~clp, j, n); j < e; ++j) step(j, std::integral_constant<int, 3 | X>{});
        for (const int e = next_set(rin | ~clp, j, n); j < e; ++j) step(j, std::integral_constant<int, 2 | X>{});
    }
}

// Square test of one pixel: its column (c.inx) and, unless the square holds
// every row of the tile (ROWS_IN), its row.
template <bool ROWS_IN>
__device__ __forceinline__ bool square_test(const Splat& s, const ColTerm& c, int py) {
    return ROWS_IN ? c.inx : (c.inx && py >= s.y0 && py <= s.y1);
}

// Lane layout (adjoint): a 16 x 16 tile is one wave, every lane holding four
// pixels (rows r, r + 4, r + 8, r + 12 of its column); 8 x 8 is one wave with one
// pixel per lane; 32 x 32 is four waves with four pixels per lane.  The per-splat
// LDS reads, loop control and cross-lane reductions are shared by all of a
// lane's pixels.
template <int B>
struct Shape {
    static constexpr int NT = (B == 32) ? 256 : 64;  // threads per tile
    static constexpr int PPL = B * B / NT;           // pixels per lane
};
// SPLIT: the forward spreads a 16 x 16 tile over two waves (two pixels per
// lane, rows r and r + 8 of a column).  When all of a launch's tiles are
// resident at once, the launch ends with its longest tile, and halving the
// longest unit of work outweighs sharing the column terms over two pixels
// instead of four (one view: 0.128 -> 0.122 ms; one pixel per lane: 0.155 ms).
// Launches of many more tiles than wave slots balance themselves and only pay
// the extra instructions (32 views: 5.0 -> 5.8 ms), so they keep one wave per
// tile.  The adjoint keeps one wave per tile: its tiles are dispatched longest
// first, and two waves would double its atomics.
template <int B, bool SPLIT>
struct ShapeF {
    static constexpr int NT = (B == 16 && SPLIT) ? 128 : Shape<B>::NT;
    static constexpr int PPL = B * B / NT;
};
// at most this many tiles in a launch take the split forward (about one wave
// slot per tile at the forward's 8 waves per SIMD)
constexpr int kSplitTiles = 8192;

// Sum over the wave (measurement counters only).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += (unsigned long long)__shfl_xor((long long)v, off);
    return v;
}

// Largest value over the wave.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    return v;
}
// Smallest value over the wave.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off));
    return v;
}

// Tile (relative to the launch's first) of this workgroup: order[blockIdx.x]
// when an order is given (the launch's tiles by decreasing cost, so that the
// expensive tiles start first and every SIMD receives a mix of costs; an entry
// out of range, which a permutation never has, falls back to blockIdx.x).
__device__ __forceinline__ int dispatch_tile(const uint32_t* __restrict__ order) {
    const uint32_t b = blockIdx.x;
    if (!order) return (int)b;
    const uint32_t t = order[b];
    return (int)(t < gridDim.x ? t : b);
}

// STATS = true is a measurement-only instantiation that also counts (pixel,
// splat) evaluations and blends into counters[0..1].  tcost[tile] receives
// the tile's last contributor (the adjoint's work on it), thist[cost_bucket]
// counts the launch's tiles per bucket.
// Waves per SIMD the forward asks registers for: with one or two pixels per
// lane, 8 (at most 64 registers, about 1 % faster than the 7 the compiler
// would otherwise settle for); with four, the blending state of four pixels
// stays live across the list walk, and 6 (5 with the merging walk) avoids
// spilling it (32 views: 6.5 -> 5.9 ms).
template <int B, bool SPLIT, bool MERGE>
struct FwdWaves {
    static constexpr int value = ShapeF<B, SPLIT>::PPL == 4 ? (MERGE ? 5 : 6) : 8;
};
// Pulls the next chunk of the tile's list (up to `need` entries) into s_ids and
// its length into *s_cnt; called by the first wave only.
template <bool MERGE, int CHUNK>
__device__ __forceinline__ int walk_chunk(TileWalk<MERGE>& walk, WalkQueues& q, uint32_t* s_ids, int* s_cnt,
                                          int need) {
    const int lane = __lane_id();
    int cnt = 0;
    for (int c0 = 0; c0 < need; c0 += 64) {
        uint32_t id;
        const int got = walk.next(min(64, need - c0), q, id);
        if (lane < got) s_ids[c0 + lane] = id;
        cnt += got;
        if (got < min(64, need - c0)) break;  // the list ended (wave-uniform)
    }
    if (lane == 0) *s_cnt = cnt;
    return cnt;
}

// MERGE: the tile's list merges the static group's 3D list with the view's 4D
// list (shared static binning); otherwise it is one list.
template <int B, int CHUNK, bool STATS, bool SPLIT, bool MERGE>
__global__ void __launch_bounds__((ShapeF<B, SPLIT>::NT), (FwdWaves<B, SPLIT, MERGE>::value)) k_composite_fwd(
    const Rec* __restrict__ recs, int N, CoarseLists lists, const ViewParams* __restrict__ views, int v0, int v1,
    const uint32_t* __restrict__ order, PtrTable images, float* __restrict__ Tfin, uint32_t* __restrict__ ncontrib,
    float* __restrict__ Cout, uint32_t* __restrict__ tcost, uint32_t* __restrict__ thist, uint32_t* __restrict__ tids,
    unsigned long long* counters) {
    constexpr int NT = ShapeF<B, SPLIT>::NT, PPL = ShapeF<B, SPLIT>::PPL;
    // two waves per tile: wave 0 walks the next chunk's entries while wave 1
    // stages the current chunk's records (the ids double-buffered); one wave
    // walks and then stages
    constexpr bool AHEAD = NT > 64;
    __shared__ LSplat s_sp[CHUNK];
    __shared__ uint32_t s_ids[AHEAD ? 2 : 1][CHUNK];
    __shared__ WalkQueues s_q;
    __shared__ int s_cnt[2];
    __shared__ uint32_t s_cost;
    const int gt = views[v0].tile_base + dispatch_tile(order);
    const int view = find_view_of_tile(views, v0, v1, gt);
    const ViewParams& V = views[view];
    const int tile = gt - V.tile_base;
    float* __restrict__ image = images.p[view];
    const int tx = tile % V.tiles_x, ty = tile / V.tiles_x;
    TileWalk<MERGE> walk;
    walk.init(lists, V, view, recs, N, super_factor(B), tx, ty);
    // all pixels of a lane share one column (NT is a multiple of B)
    const int px = tx * B + (int)threadIdx.x % B;
    const float pxc = (float)px + 0.5f;
    int py[PPL];
    // A finished pixel (and one outside the image) has its row centre pyc at
    // +inf: its offset dy to any splat is +inf, the power -inf (the scaled
    // conic entry qc is negative), so that no later pair passes the blending
    // test and the pixel needs no test of its own; T keeps its final
    // transmittance.
    float pyc[PPL], T[PPL], cr[PPL], cg[PPL], cb[PPL];
    uint32_t last[PPL];
    bool lane_done = true;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int p = (int)threadIdx.x + k * NT;
        py[k] = ty * B + p / B;
        const bool inside = px < V.W && py[k] < V.H;
        pyc[k] = inside ? (float)py[k] + 0.5f : __builtin_inff();
        T[k] = 1.0f;
        cr[k] = cg[k] = cb[k] = 0.f;
        last[k] = 0u;
        lane_done = lane_done && !inside;
    }
    unsigned long long n_eval = 0, n_blend = 0;
    // wave-uniform: the splat loop runs for the whole wave (finished pixels are
    // masked), so that its per-pixel flags stay lane masks
    bool wave_done = __ballot(!lane_done) == 0ull;
    const int tid = (int)threadIdx.x;
    uint32_t rel0 = 0;    // list position of the chunk's first entry
    uint32_t walked = 0;  // entries walked (wave 0)
    int cur = 0;          // the chunk's id buffer
    if (AHEAD && tid < 64) walked += (uint32_t)walk_chunk<MERGE, CHUNK>(walk, s_q, s_ids[0], &s_cnt[0], CHUNK);
    for (;;) {
        if (__syncthreads_count(wave_done) == NT) break;
        if (!AHEAD) {
            if (tid < 64) walked += (uint32_t)walk_chunk<MERGE, CHUNK>(walk, s_q, s_ids[0], &s_cnt[0], CHUNK);
            __syncthreads();
        }
        const int cnt = s_cnt[cur];
        if (cnt == 0) break;  // uniform: the list is exhausted
        if (AHEAD && tid < 64) {
            if (cnt == CHUNK) {
                walked += (uint32_t)walk_chunk<MERGE, CHUNK>(walk, s_q, s_ids[cur ^ 1], &s_cnt[cur ^ 1], CHUNK);
            } else if (tid == 0) {
                s_cnt[cur ^ 1] = 0;  // the list ended inside this chunk
            }
        } else {
            constexpr int NS = AHEAD ? NT - 64 : NT;  // staging threads
            for (int k = AHEAD ? tid - 64 : tid; k < cnt; k += NS) {
                const uint32_t raw = s_ids[cur][k];
                stage_splat(walk.record(raw), raw & ~kFromStatic, ty * B, ty * B + B - 1, s_sp[k]);
                // the list's head, kept for the adjoint
                if (tids && rel0 + (uint32_t)k < (uint32_t)kTileIds) tids[(size_t)gt * kTileIds + rel0 + k] = raw;
            }
        }
        __syncthreads();
        if (!wave_done) {
            // one blending step of the lane's pixels with splat j; true once every
            // pixel of the wave is finished
            auto step = [&](int j, auto rows_tag) {
                constexpr bool RI = decltype(rows_tag)::value;
                const Splat s = to_splat(s_sp[j]);
                const ColTerm c = eval_col(s, px, pxc);
                // lanes with a pixel whose transmittance would fall below the
                // floor: a pixel finishes only at such a step
                unsigned long long near = 0ull;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    float dy, G, alpha;
                    bool clamped;
                    const bool in = square_test<RI>(s, c, py[k]);
                    const bool ok = eval_pix(s, c, in, pyc[k], dy, G, alpha, clamped);  // (false once finished)
                    const float Tn = next_T(T[k], alpha);
                    const bool low = Tn < kMinT;
                    near |= __builtin_amdgcn_ballot_w64(low);
                    const bool stop = ok && low;
                    const bool bl = ok && !stop;
                    const float w = bl ? alpha * T[k] : 0.0f;
                    cr[k] = __builtin_fmaf(s.cr, w, cr[k]);
                    cg[k] = __builtin_fmaf(s.cg, w, cg[k]);
                    cb[k] = __builtin_fmaf(s.cb, w, cb[k]);
                    if (STATS) {
                        n_eval += (pyc[k] < __builtin_inff() && in) ? 1u : 0u;
                        n_blend += bl ? 1u : 0u;
                    }
                    T[k] = bl ? Tn : T[k];
                    pyc[k] = stop ? __builtin_inff() : pyc[k];
                    last[k] = bl ? rel0 + (uint32_t)j + 1u : last[k];
                }
                if (near == 0ull) return false;  // wave-uniform: no pixel finished here
                bool act = false;
#pragma unroll
                for (int k = 0; k < PPL; ++k) act = act || pyc[k] < __builtin_inff();
                return __ballot(act) == 0ull;
            };
            // splats whose square holds all of the tile's rows take the step
            // without the row test
            for (int g0 = 0; g0 < cnt && !wave_done; g0 += 64) {
                const int gn = min(64, cnt - g0);
                wave_done = walk_runs(rows_in_mask(s_sp, g0, gn), gn,
                                      [&](int i, auto tag) { return step(g0 + i, tag); });
            }
        }
        rel0 += (uint32_t)cnt;
        if (AHEAD) cur ^= 1;
    }
    const size_t HW = (size_t)V.W * V.H;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        if (px < V.W && py[k] < V.H) {
            const size_t p = (size_t)py[k] * V.W + px;
            const float Tk = T[k];
            const float o0 = __builtin_fmaf(Tk, V.bg[0], cr[k]), o1 = __builtin_fmaf(Tk, V.bg[1], cg[k]),
                        o2 = __builtin_fmaf(Tk, V.bg[2], cb[k]);
            image[p] = o0;
            image[HW + p] = o1;
            image[2 * HW + p] = o2;
            if (Tfin) {  // the adjoint's per-pixel state (not kept by an inference render)
                const size_t q = (size_t)V.pix_base + p;
                Tfin[q] = Tk;
                ncontrib[q] = last[k];
                Cout[3 * (size_t)V.pix_base + p] = o0;
                Cout[3 * (size_t)V.pix_base + HW + p] = o1;
                Cout[3 * (size_t)V.pix_base + 2 * HW + p] = o2;
            }
        }
    }
    // the tile's cost for the adjoint: its last contributor over all pixels
    // (tcost is the same for the whole launch, so the barriers below stay uniform)
    if (tcost) {
    uint32_t lane_last = 0u;
#pragma unroll
    for (int k = 0; k < PPL; ++k) lane_last = max(lane_last, last[k]);
    const uint32_t wave_last = wave_max_u32(lane_last);
    uint32_t tile_last = wave_last;
    if (NT == 64) {
        if (threadIdx.x == 0) {
            tcost[gt] = wave_last;
            atomicAdd(&thist[cost_bucket(wave_last)], 1u);
        }
    } else {
        if (threadIdx.x == 0) s_cost = 0u;
        __syncthreads();
        if (__lane_id() == 0) atomicMax(&s_cost, wave_last);
        __syncthreads();
        tile_last = s_cost;
        if (threadIdx.x == 0) {
            tcost[gt] = s_cost;
            atomicAdd(&thist[cost_bucket(s_cost)], 1u);
        }
    }
    if (STATS && threadIdx.x < 64) {
        // the tile's list length: the entries walked and those left
        const unsigned long long len = (unsigned long long)walked + walk.remaining();
        if (threadIdx.x == 0) {
            atomicAdd(&counters[4], len);
            atomicAdd(&counters[5], (unsigned long long)tile_last);
        }
    }
    }
    if (STATS) {
        const unsigned long long e = wave_sum_u64(n_eval), b = wave_sum_u64(n_blend);
        if (__lane_id() == 0) {
            atomicAdd(&counters[0], e);
            atomicAdd(&counters[1], b);
        }
    }
}

// Cross-lane building blocks of the backward's reduction (gfx950).
// swap32_add(a, b): lanes 0-31 get a[l] + a[l + 32], lanes 32-63 get b[l - 32] + b[l].
__device__ __forceinline__ float swap32_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// swap16_add(a, b): with rows of 16 lanes, row 0 gets a.r0 + a.r1, row 1 b.r0 + b.r1,
// row 2 a.r2 + a.r3, row 3 b.r2 + b.r3 (lane by lane within the rows).
__device__ __forceinline__ float swap16_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// Wave sums of nine values by reduce-scatter: after two swap levels two
// registers hold, per 16-lane row, one value summed over 4 lanes (e0 e2 e1 e3
// and e4 e6 e5 e7 by row); two more levels inside the rows (mirror, half-row
// mirror, the second also taking e8) leave one register, whose quad sums
// finish the row sums.  Result layout in each row r: lanes 0-3 the row's first
// value (e0 e2 e1 e3 for r = 0 1 2 3), lanes 8-11 its second (e4 e6 e5 e7),
// lanes 4-7 the row's part of e8 (the sum of e8 over its 16 lanes).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_sum9(float e0, float e1, float e2, float e3, float e4, float e5, float e6,
                                           float e7, float e8) {
    const float f0 = swap32_add(e0, e1), f1 = swap32_add(e2, e3), f2 = swap32_add(e4, e5), f3 = swap32_add(e6, e7);
    const float g0 = swap16_add(f0, f1), g1 = swap16_add(f2, f3);
    // row mirror: lanes 0-7 pair g0 with lanes 15-8, lanes 8-15 g1 (each half
    // of the row written by its own DPP add, the other half's banks masked
    // off); e8 in all lanes
    float x;
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %1, %1 row_mirror row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %0, %2, %2 row_mirror row_mask:0xf bank_mask:0xc"
        : "=&v"(x)
        : "v"(g0), "v"(g1));
    const float y = e8 + dpp_f<0x140>(e8);
    // half-row mirror: lanes 0-3 (8-11) pair x with lanes 7-4 (15-12), lanes 4-7 (12-15) y
    float z;
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %1, %1 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
        "v_add_f32_dpp %0, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xa"
        : "=&v"(z)
        : "v"(x), "v"(y));
    z += dpp_f<0x4E>(z);  // quad lane ^ 2
    z += dpp_f<0xB1>(z);  // quad lane ^ 1
    return z;
}

// Per splat of the tile's list (up to its last contributor), the wave's nine
// gradient sums (wave_sum9) are added into the splat's g2 record with one
// global atomic instruction (twelve lanes, one record).
// static_rows (MERGE): the gradients of the static list's entries go to the
// records of the static group's view.
// (registers for 5 waves per SIMD, what the plain adjoint uses anyway: the
// merging walk would otherwise take the occupancy down to 4)
template <int B, int CHUNK, bool STATS, bool MERGE>
__global__ void __launch_bounds__(Shape<B>::NT, 5) k_composite_bwd(
    const Rec* __restrict__ recs, int N, CoarseLists lists, int static_rows, const ViewParams* __restrict__ views,
    int v0, int v1, const uint32_t* __restrict__ order, CPtrTable dls, const float* __restrict__ Tfin,
    const uint32_t* __restrict__ ncontrib, const float* __restrict__ Cout, const uint32_t* __restrict__ tids,
    float* __restrict__ g2, unsigned long long* counters) {
    constexpr int NT = Shape<B>::NT, PPL = Shape<B>::PPL;
    __shared__ LSplat s_sp[CHUNK];
    __shared__ uint32_t s_ids[CHUNK];
    __shared__ WalkQueues s_q;
    __shared__ int s_cnt;
    __shared__ uint32_t s_max;
    const int gt = views[v0].tile_base + dispatch_tile(order);
    const int view = find_view_of_tile(views, v0, v1, gt);
    const ViewParams& V = views[view];
    const int tile = gt - V.tile_base;
    // indexed by splat id: the view's own gradient records, and those its
    // static list's entries go to
    float* __restrict__ g2s = g2 + (size_t)(MERGE && static_rows ? V.static_view : view) * N * kG2Stride;
    g2 += (size_t)view * N * kG2Stride;
    const float* __restrict__ dl = dls.p[view];
    const int tx = tile % V.tiles_x, ty = tile / V.tiles_x;
    TileWalk<MERGE> walk;
    walk.init(lists, V, view, recs, N, super_factor(B), tx, ty);
    const size_t HW = (size_t)V.W * V.H;
    const int lane = __lane_id();
    // all pixels of a lane share one column (NT is a multiple of B)
    const int px = tx * B + (int)threadIdx.x % B;
    const float pxc = (float)px + 0.5f;
    int py[PPL];
    float pyc[PPL], G0[PPL], G1[PPL], G2[PPL], R[PPL], T[PPL];
    uint32_t nc[PPL];
    uint32_t lane_nc = 0, lane_min = 0xFFFFFFFFu;  // (the latter over the pixels inside the image)
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int p = (int)threadIdx.x + k * NT;
        py[k] = ty * B + p / B;
        pyc[k] = (float)py[k] + 0.5f;
        G0[k] = G1[k] = G2[k] = R[k] = 0.f;
        nc[k] = 0u;
        if (px < V.W && py[k] < V.H) {
            const size_t q = (size_t)py[k] * V.W + px;
            G0[k] = dl[q]; G1[k] = dl[HW + q]; G2[k] = dl[2 * HW + q];
            const float c0 = Cout[3 * (size_t)V.pix_base + q];
            const float c1 = Cout[3 * (size_t)V.pix_base + HW + q];
            const float c2 = Cout[3 * (size_t)V.pix_base + 2 * HW + q];
            R[k] = G0[k] * c0 + G1[k] * c1 + G2[k] * c2;  // dot(dL/dC, C_out)
            nc[k] = ncontrib[(size_t)V.pix_base + q];
            lane_min = min(lane_min, nc[k]);
        }
        T[k] = 1.0f;
        lane_nc = max(lane_nc, nc[k]);
    }
    if (threadIdx.x == 0) s_max = 0u;
    __syncthreads();
    if (lane_nc) atomicMax(&s_max, lane_nc);
    __syncthreads();
    // the forward's last contributor (the walk ends with the tile's list, so a
    // state whose per-pixel part comes from another forward reads no foreign
    // entries)
    const uint32_t total = s_max;
    const uint32_t wave_nc = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_max_u32(lane_nc));
    // entries before the smallest last contributor of the wave's pixels in the
    // image have every pixel live; pixels outside the image have no upstream
    // gradient and R = 0, so that their terms are exact zeros in any case
    const uint32_t wave_min = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_min_u32(lane_min));
    unsigned long long n_eval = 0, n_blend = 0;
    // after wave_sum9, lane 16 r holds component 0 2 1 3 (r = 0 1 2 3) of g2,
    // lane 16 r + 8 component 4 6 5 7, lane 16 r + 4 row r's part of
    // component 8, which goes to slot 8 + r of the record (the four parts are
    // summed where the record is read).  One atomic instruction of these
    // twelve lanes adds them to the splat's record, no two to one address.  The
    // centre and conic slots hold their sums without the constant factors and
    // the splat's opacity, which the projection adjoint applies where it reads
    // the record (once per record instead of once per tile).
    const int row = lane >> 4, lr = lane & 15;
    const int comp0 = ((row & 1) << 1) | (row >> 1);
    const bool alane = lr == 0 || lr == 4 || lr == 8;
    const int comp = lr == 0 ? comp0 : (lr == 8 ? 4 + comp0 : 8 + row);
    const uint32_t comp_off = (uint32_t)comp * (uint32_t)sizeof(float);  // bytes into the record
    // raw buffer resources over the records (no range limit; data format 32
    // bits, the gfx9 word 3): record offsets stay below 2^32 bytes per view
    const __amdgpu_buffer_rsrc_t g2_rsrc = __builtin_amdgcn_make_buffer_rsrc(g2, (short)0, -1, 0x00020000);
    const __amdgpu_buffer_rsrc_t g2s_rsrc = __builtin_amdgcn_make_buffer_rsrc(g2s, (short)0, -1, 0x00020000);
    const int tid = (int)threadIdx.x;
    // the forward kept the list's head: a tile whose contributors all lie in
    // it reads them from there, any other walks its list again
    const bool kept = total <= (uint32_t)kTileIds;
    const uint32_t* __restrict__ head = tids + (size_t)gt * kTileIds;
    for (uint32_t rel0 = 0; rel0 < total;) {
        __syncthreads();  // the previous chunk's LDS is no longer read
        int cnt;
        if (kept) {
            cnt = (int)min((uint32_t)CHUNK, total - rel0);
        } else {
            if (tid < 64) walk_chunk<MERGE, CHUNK>(walk, s_q, s_ids, &s_cnt, (int)min((uint32_t)CHUNK, total - rel0));
            __syncthreads();
            cnt = s_cnt;
            if (cnt == 0) break;  // uniform: the list is exhausted
        }
        for (int k = tid; k < cnt; k += NT) {
            uint32_t raw = kept ? head[rel0 + k] : s_ids[k];
            // (a head written by another forward reads no record past the set)
            if ((MERGE ? (raw & ~kFromStatic) : raw) >= (uint32_t)N) raw = 0u;
            stage_splat(walk.record(raw), raw, ty * B, ty * B + B - 1, s_sp[k]);  // (gid keeps the static flag)
        }
        __syncthreads();
        // entries past this wave's last contributor need no work
        const int jend = wave_nc > rel0 ? (int)min((uint32_t)cnt, wave_nc - rel0) : 0;
        // the adjoint of one blending step with splat j; gid: its splat id
        // tag bit 0: the square holds every row of the tile; bit 1: the splat's
        // opacity may reach the 0.99 clamp
        auto step = [&](int j, uint32_t gid, auto tag) {
            constexpr bool RI = (decltype(tag)::value & 1) != 0;
            constexpr bool CL = (decltype(tag)::value & 2) != 0;
            constexpr bool AL = (decltype(tag)::value & 4) != 0;  // every pixel live
            float qa2, qc2;
            const Splat s = to_splat_wide(s_sp[j], qa2, qc2);
            const ColTerm c = eval_col(s, px, pxc);
            // per-splat sums of this lane's pixels: dL/dopacity, dL/drgb, and the
            // moments sum q, sum q dy, sum q dy^2 of q = dL/dalpha * exp2(power),
            // which is dL/dpower (natural log domain) divided by the splat's opacity
            // (the lane's pixels share dx, so the centre and conic terms follow
            // from them below)
            float e5 = 0.f, e6 = 0.f, e7 = 0.f, e8 = 0.f, sdy = 0.f, syy = 0.f;
            bool any = false;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                float dy, Gk, alpha;
                bool clamped;
                const bool live = AL || rel0 + (uint32_t)j < nc[k];
                const bool in = square_test<RI>(s, c, py[k]);
                const bool pass = eval_pix(s, c, in, pyc[k], dy, Gk, alpha, clamped);
                const bool ok = pass && live;
                if (STATS) {
                    n_eval += (live && in) ? 1u : 0u;
                    n_blend += ok ? 1u : 0u;
                }
                any = any || ok;
                const float a = ok ? alpha : 0.0f;
                const float w = a * T[k];
                const float gc = G0[k] * s.cr + G1[k] * s.cg + G2[k] * s.cb;
                R[k] = __builtin_fmaf(-w, gc, R[k]);  // less the colour blended so far
                // dL/dalpha = T dot(dL/dC, c) - dot(dL/dC, colour behind) / (1 - alpha),
                // colour behind = C_out - prefix, whose dot product R now holds
                // (it includes T_final * bg)
                const float ioma = __builtin_amdgcn_rcpf(1.0f - alpha);
                const float da = __builtin_fmaf(T[k], gc, -(R[k] * ioma));
                e6 = __builtin_fmaf(G0[k], w, e6);
                e7 = __builtin_fmaf(G1[k], w, e7);
                e8 = __builtin_fmaf(G2[k], w, e8);
                // no gradient through the 0.99 clamp (da is finite: alpha <= 0.99)
                const float gz = (ok && !(CL && clamped)) ? Gk : 0.0f;
                const float q = da * gz;  // dL/dopacity share; dL/dpower = opacity * q
                const float qdy = q * dy;
                e5 += q;
                sdy += qdy;
                syy = __builtin_fmaf(qdy, dy, syy);
                T[k] = next_T(T[k], a);  // unchanged where a = 0
            }
            // conic and centre terms without their constant factors and the
            // opacity (applied after the reduction): sum q (2 qa dx + qb dy),
            // sum q (qb dx + 2 qc dy), sum q dx^2, sum q dx dy, sum q dy^2,
            // from A = dx sum q
            const float A = c.dx * e5;
            const float e0 = __builtin_fmaf(qa2, A, s.qb * sdy);
            const float e1 = __builtin_fmaf(s.qb, A, qc2 * sdy);
            const float e2 = c.dx * A, e3 = c.dx * sdy, e4 = syy;
            if (__builtin_amdgcn_ballot_w64(any) != 0ull) {  // wave-uniform: reduce only when some lane blended
                const float h = wave_sum9(e0, e1, e2, e3, e4, e5, e6, e7, e8);
                // the cross-lane operations need the whole wave: consume their
                // result here, before the lane-divergent atomic below
                asm volatile("" ::"v"(h));
                if (alane) {
                    // buffer atomic: the view's records as the resource, the
                    // record's offset (scalar) and the lane's slot (vector) added
                    // by the address unit
                    __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(
                        h, (MERGE && (gid & kFromStatic)) ? g2s_rsrc : g2_rsrc, (int)comp_off,
                        (int)((gid & ~kFromStatic) * (uint32_t)(kG2Stride * sizeof(float))), 0);
                }
            }
        };
        // splats whose square holds all of the tile's rows take the step without
        // the row test, those whose opacity stays below the clamp without the
        // clamp test; in the merging launches (many more tiles than wave slots,
        // bound by instruction throughput) those before the wave's smallest last
        // contributor also without the live test (a single view's launch, bound
        // by its longest tiles, ran 2 % slower with the extra variants; the
        // counting instances keep the test, whose counts include it); the
        // group's splat ids sit one per lane and reach the step as wave-uniform
        // values
        for (int g0 = 0; g0 < jend; g0 += 64) {
            const int gn = min(64, jend - g0);
            const uint32_t gids = s_sp[g0 + min(lane, gn - 1)].gid;
            const unsigned long long rin = rows_in_mask(s_sp, g0, gn), clp = clamp_mask(s_sp, g0, gn);
            const auto run = [&](int i, auto tag) {
                step(g0 + i, (uint32_t)__builtin_amdgcn_readlane((int)gids, i), tag);
            };
            if constexpr (MERGE && !STATS) {
                const int jall =
                    (int)max((int64_t)0, min((int64_t)gn, (int64_t)wave_min - (int64_t)(rel0 + (uint32_t)g0)));
                walk_runs2<4>(rin, clp, 0, jall, run);
                walk_runs2<0>(rin, clp, jall, gn, run);
            } else {
                walk_runs2<0>(rin, clp, 0, gn, run);
            }
        }
        rel0 += (uint32_t)cnt;
    }
    if (STATS) {
        const unsigned long long e = wave_sum_u64(n_eval), b = wave_sum_u64(n_blend);
        if (__lane_id() == 0) {
            atomicAdd(&counters[2], e);
            atomicAdd(&counters[3], b);
        }
    }
}

bool composite_supported(int tile, int chunk) {
    return (tile == 8 || tile == 16 || tile == 32) && (chunk == 64 || chunk == 128 || chunk == 256 || chunk == 512);
}

template <class T>
struct same_type {
    using type = T;
};
// Launches k on st; with events, through the dispatch-timestamp launch so that
// e0 / e1 take the kernel's own start and end (no extra commands on the stream).
template <typename... P>
static void launch_timed(void (*k)(P...), int grid, int block, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                         typename same_type<P>::type... args) {
    if (!e0 && !e1) {
        k<<<grid, block, 0, st>>>(args...);
        return;
    }
    void* a[] = {(void*)&args...};
    (void)hipExtLaunchKernel((const void*)k, dim3(grid), dim3(block), a, 0, st, e0, e1, 0);
}

template <int B, int C>
static void fwd_t(const Rec* recs, int N, const CoarseLists& lists, bool merge, const ViewParams* views, int v0,
                  int v1, int n_tiles, const uint32_t* order, const PtrTable& images, float* Tfin,
                  uint32_t* ncontrib, float* Cout, uint32_t* tcost, uint32_t* thist, uint32_t* tids,
                  unsigned long long* counters, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const bool stats = counters != nullptr;
#define H4D_FWD(SPLIT)                                                                                            \
    launch_timed(merge ? (stats ? k_composite_fwd<B, C, true, SPLIT, true> : k_composite_fwd<B, C, false, SPLIT, true>) \
                       : (stats ? k_composite_fwd<B, C, true, SPLIT, false>                                         \
                                : k_composite_fwd<B, C, false, SPLIT, false>),                                      \
                 n_tiles, ShapeF<B, SPLIT>::NT, st, e0, e1, recs, N, lists, views, v0, v1, order, images, Tfin,    \
                 ncontrib, Cout, tcost, thist, tids, counters)
    if constexpr (B == 16) {
        if (n_tiles <= kSplitTiles) {
            H4D_FWD(true);
            return;
        }
    }
    H4D_FWD(false);
#undef H4D_FWD
}
template <int B, int C>
static void bwd_t(const Rec* recs, int N, const CoarseLists& lists, bool merge, int static_rows,
                  const ViewParams* views, int v0, int v1, int n_tiles, const uint32_t* order, const CPtrTable& dls,
                  const float* Tfin, const uint32_t* ncontrib, const float* Cout, const uint32_t* tids, float* g2,
                  unsigned long long* counters, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    constexpr int NT = Shape<B>::NT;
    const bool stats = counters != nullptr;
    launch_timed(merge ? (stats ? k_composite_bwd<B, C, true, true> : k_composite_bwd<B, C, false, true>)
                       : (stats ? k_composite_bwd<B, C, true, false> : k_composite_bwd<B, C, false, false>),
                 n_tiles, NT, st, e0, e1, recs, N, lists, static_rows, views, v0, v1, order, dls, Tfin, ncontrib,
                 Cout, tids, g2, counters);
}

// Tile lists written out (for inspection): one wave per tile walks the list as
// the blending kernels do.  k_walk_count: cnt[tile] = list length;
// k_walk_dump: the splat ids of tile t (indices into the merged set [4D | 3D])
// at out[offsets[t] ..), and ranges[t] = [offsets[t], offsets[t] + cnt[t]).
template <int S, bool MERGE>
__global__ void __launch_bounds__(64) k_walk_count(const Rec* __restrict__ recs, int N, CoarseLists lists,
                                                   const ViewParams* __restrict__ views, int v0, int v1,
                                                   uint32_t* __restrict__ cnt) {
    __shared__ WalkQueues s_q;
    const int gt = views[v0].tile_base + (int)blockIdx.x;
    const int view = find_view_of_tile(views, v0, v1, gt);
    const ViewParams& V = views[view];
    const int tile = gt - V.tile_base;
    TileWalk<MERGE> walk;
    walk.init(lists, V, view, recs, N, S, tile % V.tiles_x, tile / V.tiles_x);
    const uint64_t n = walk.remaining();
    if (threadIdx.x == 0) cnt[blockIdx.x] = (uint32_t)n;
}

template <int S, bool MERGE>
__global__ void __launch_bounds__(64) k_walk_dump(const Rec* __restrict__ recs, int N, CoarseLists lists,
                                                  const ViewParams* __restrict__ views, int v0, int v1,
                                                  const unsigned long long* __restrict__ offsets,
                                                  uint32_t* __restrict__ out, uint64_t out_cap,
                                                  int64_t* __restrict__ ranges) {
    __shared__ WalkQueues s_q;
    const int gt = views[v0].tile_base + (int)blockIdx.x;
    const int view = find_view_of_tile(views, v0, v1, gt);
    const ViewParams& V = views[view];
    const int tile = gt - V.tile_base;
    TileWalk<MERGE> walk;
    walk.init(lists, V, view, recs, N, S, tile % V.tiles_x, tile / V.tiles_x);
    const unsigned long long o0 = offsets[blockIdx.x], o1 = offsets[blockIdx.x + 1];
    unsigned long long o = o0;
    for (;;) {
        uint32_t id;
        const int got = walk.next(64, s_q, id);
        const unsigned long long w = o + (unsigned)__lane_id();
        if (__lane_id() < got && w < o1 && w < out_cap) out[w] = id & ~kFromStatic;
        o += (unsigned)got;
        if (got < 64) break;
    }
    if (threadIdx.x == 0) {
        ranges[2 * (size_t)gt] = (int64_t)o0;
        ranges[2 * (size_t)gt + 1] = (int64_t)o1;
    }
}

void launch_walk_lists(int tile, const Rec* recs, int N, const CoarseLists& lists, bool merge,
                       const ViewParams* views, int v0, int v1, int n_tiles, uint32_t* cnt,
                       unsigned long long* offsets, unsigned long long* partials, uint32_t* out, uint64_t out_cap,
                       int64_t* ranges, hipStream_t st) {
    if (n_tiles == 0) return;
#define H4D_WALK(S, M)                                                                                       \
    do {                                                                                                     \
        k_walk_count<S, M><<<n_tiles, 64, 0, st>>>(recs, N, lists, views, v0, v1, cnt);                      \
        launch_scan_u32_u64(cnt, nullptr, n_tiles, offsets, partials, st);                                   \
        k_walk_dump<S, M><<<n_tiles, 64, 0, st>>>(recs, N, lists, views, v0, v1, offsets, out, out_cap,      \
                                                  ranges);                                                 \
    } while (0)
    if (super_factor(tile) == 2) {
        if (merge) H4D_WALK(2, true); else H4D_WALK(2, false);
    } else {
        if (merge) H4D_WALK(4, true); else H4D_WALK(4, false);
    }
#undef H4D_WALK
}

#define H4D_DISPATCH(FN, ...)                                                   \
    do {                                                                        \
        if (tile == 8 && chunk == 64) FN<8, 64>(__VA_ARGS__);                   \
        else if (tile == 16 && chunk == 64) FN<16, 64>(__VA_ARGS__);            \
        else if (tile == 32 && chunk == 64) FN<32, 64>(__VA_ARGS__);            \
        else if (tile == 8 && chunk == 128) FN<8, 128>(__VA_ARGS__);            \
        else if (tile == 8 && chunk == 256) FN<8, 256>(__VA_ARGS__);            \
        else if (tile == 8 && chunk == 512) FN<8, 512>(__VA_ARGS__);            \
        else if (tile == 16 && chunk == 128) FN<16, 128>(__VA_ARGS__);          \
        else if (tile == 16 && chunk == 256) FN<16, 256>(__VA_ARGS__);          \
        else if (tile == 16 && chunk == 512) FN<16, 512>(__VA_ARGS__);          \
        else if (tile == 32 && chunk == 128) FN<32, 128>(__VA_ARGS__);          \
        else if (tile == 32 && chunk == 256) FN<32, 256>(__VA_ARGS__);          \
        else if (tile == 32 && chunk == 512) FN<32, 512>(__VA_ARGS__);          \
    } while (0)

void launch_composite_fwd(int tile, int chunk, const Rec* recs, int N, const CoarseLists& lists, bool merge,
                          const ViewParams* views, int v0, int v1, int n_tiles, const uint32_t* order,
                          const PtrTable& images, float* Tfin, uint32_t* ncontrib, float* Cout, uint32_t* tcost,
                          uint32_t* thist, uint32_t* tids, unsigned long long* counters, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1) {
    if (n_tiles == 0) return;
    H4D_DISPATCH(fwd_t, recs, N, lists, merge, views, v0, v1, n_tiles, order, images, Tfin, ncontrib, Cout, tcost,
                 thist, tids, counters, st, e0, e1);
}

void launch_composite_bwd(int tile, int chunk, const Rec* recs, int N, const CoarseLists& lists, bool merge,
                          int static_rows, const ViewParams* views, int v0, int v1, int n_tiles,
                          const uint32_t* order, const CPtrTable& dls, const float* Tfin, const uint32_t* ncontrib,
                          const float* Cout, const uint32_t* tids, float* g2, unsigned long long* counters,
                          hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (n_tiles == 0) return;
    H4D_DISPATCH(bwd_t, recs, N, lists, merge, static_rows, views, v0, v1, n_tiles, order, dls, Tfin, ncontrib,
                 Cout, tids, g2, counters, st, e0, e1);
}

}  // namespace h4d

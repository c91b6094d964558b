// Tile-list walk: the depth-ordered splats of one tile (Alg. 1, the list that
// BlendInOrder traverses), read straight from the sorted coarse lists.
//
// Binning leaves, per super-tile, a list of coarse entries sorted by (depth
// bits, id): key = super-tile id | tile mask << 16, value = splat id.  A tile's
// list is the sub-sequence of its super-tile's list whose mask holds the tile.
// Instead of writing every tile's list out (most of a long list lies behind the
// point where all of the tile's pixels are saturated and is never read), the
// blending kernels pull the next entries of their tile from the coarse list on
// demand, one 64-wide window at a time: a ballot on the tile's mask bit and a
// prefix count compact the window's entries in order.
//
// Shared static binning (MERGE): the 3D Gaussians of views that repeat a
// camera are binned once per camera, so a tile's list is the depth-order merge
// of two lists - the static group's 3D entries and the view's own 4D entries.
// Each side is compacted into a queue of up to 64 entries (with their records'
// depth keys); the next up to 64
// entries of the merge come from a bitonic merge of the two queues across the
// wave.  Equal depth bits put the 4D entry first, which is the order of the
// merged index [4D | 3D] that a single sort over both sets gives.
//
// One wave walks; the state lives in its registers (positions, queue counts)
// and in its own LDS queues.
#pragma once

#include "common.hpp"

namespace h4d {

// Flag on an id taken from the static group's list: its record is in the
// group's view (static_view), not in the tile's own.
constexpr uint32_t kFromStatic = 0x80000000u;

struct WalkRun {
    int64_t pos, end;
};

// LDS of the walking wave: the two merge queues (ids, depth bits).
struct WalkQueues {
    uint32_t a[64], ad[64], b[64], bd[64];
};

__device__ __forceinline__ unsigned long long walk_lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// Appends to q[n ..) the ids of the entries of r whose key holds bit `bit`, in
// order (and, with DEPTH, their records' depth keys to qd), until n == need or r is
// exhausted; r.pos ends just past the last entry taken (or at r.end).
// Windows of 64 entries are loaded up to four at a time, as many as the
// entries still wanted suggest (about one entry in four is kept).
template <bool DEPTH>
__device__ inline int walk_fill(const CoarseLists& L, uint32_t bit, WalkRun& r, uint32_t* q, uint32_t* qd, int n,
                                int need, const Rec* __restrict__ recs) {
    const int lane = __lane_id();
    const unsigned long long lt = walk_lanemask_lt();
    while (n < need && r.pos < r.end) {
        const int64_t p0 = r.pos;
        const int nw = min(4, (need - n + 15) >> 4);
        uint32_t kk[4], vv[4], dd[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int64_t k = p0 + w * 64 + lane;
            const bool in = w < nw && k < r.end;
            kk[w] = in ? L.keys[k] : 0u;  // (a key of 0 has no tile bit)
            vv[w] = in ? L.vals[k] : 0u;
        }
#pragma unroll
        for (int w = 0; w < 4; ++w)
            if (DEPTH) dd[w] = ((kk[w] >> bit) & 1u) != 0u ? __float_as_uint(recs[vv[w]].c.w) : 0u;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if (w >= nw || n >= need || r.pos >= r.end) break;  // wave-uniform
            const bool keep = ((kk[w] >> bit) & 1u) != 0u;
            const unsigned long long m = __ballot(keep);
            const int cnt = __popcll(m);
            const int take = min(cnt, need - n);
            const int rank = __popcll(m & lt);
            if (keep && rank < take) {
                q[n + rank] = vv[w];
                if (DEPTH) qd[n + rank] = dd[w];
            }
            if (take < cnt) {
                // stop just past the lane that holds the last entry taken
                const unsigned long long last = __ballot(keep && rank == take - 1);
                r.pos = p0 + w * 64 + __builtin_ctzll(last) + 1;
            } else {
                r.pos = min(p0 + (int64_t)(w + 1) * 64, r.end);
            }
            n += take;
        }
    }
    return n;
}

// 64-bit lane exchange with lane ^ s.
__device__ __forceinline__ unsigned long long walk_xor(unsigned long long v, int s) {
    const int lo = __shfl_xor((int)(uint32_t)v, s), hi = __shfl_xor((int)(uint32_t)(v >> 32), s);
    return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Number of entries of r whose key holds `bit` (the rest of a list, for the
// counting kernels).
__device__ inline uint64_t walk_count(const CoarseLists& L, uint32_t bit, WalkRun r) {
    uint64_t c = 0;
    for (int64_t p = r.pos + __lane_id(); __ballot(p < r.end) != 0ull; p += 64) {
        const bool keep = p < r.end && ((L.keys[p] >> bit) & 1u) != 0u;
        c += (uint64_t)__popcll(__ballot(keep));
    }
    return c;
}

// Walk state of one tile.  MERGE: run a = the static group's 3D entries
// (records recs_a), run b = the view's 4D entries (records recs_b); otherwise
// run b holds the whole list.
template <bool MERGE>
struct TileWalk {
    CoarseLists L;
    uint32_t bit;
    WalkRun a, b;
    const Rec* recs_a;
    const Rec* recs_b;
    int na, nb;  // queued entries (MERGE)

    // Tile (tx, ty) of view V with S x S tiles per super-tile; recs: the
    // records of every view ([view][N]).
    __device__ void init(const CoarseLists& lists, const ViewParams& V, int view, const Rec* recs, int N, int S,
                         int tx, int ty) {
        L = lists;
        bit = 16u + (uint32_t)((ty % S) * S + (tx % S));
        const int sl = (ty / S) * V.sx + (tx / S);
        const int64_t* rb = L.ranges + 2 * (size_t)(V.super_base + sl);
        b.pos = rb[0];
        b.end = rb[1];
        recs_b = recs + (size_t)view * N;
        if (MERGE) {
            const int64_t* ra = L.ranges + 2 * (size_t)(V.static_super_base + sl);
            a.pos = ra[0];
            a.end = ra[1];
            recs_a = recs + (size_t)V.static_view * N;
        } else {
            a.pos = a.end = 0;
            recs_a = recs_b;
        }
        na = nb = 0;
    }

    // The next up to `need` (<= 64) entries: lane i receives the i-th in *id
    // (ORed with kFromStatic for an entry of the static list); returns how many
    // there are (fewer than need only at the end of the list).
    __device__ int next(int need, WalkQueues& s, uint32_t& id) {
        const int lane = __lane_id();
        if (!MERGE) {
            const int n = walk_fill<false>(L, bit, b, s.b, nullptr, 0, need, nullptr);
            id = lane < n ? s.b[lane] : 0u;
            return n;
        }
        na = walk_fill<true>(L, bit, a, s.a, s.ad, na, 64, recs_a);
        nb = walk_fill<true>(L, bit, b, s.b, s.bd, nb, 64, recs_b);
        const int k = min(need, na + nb);
        // The 64 smallest of the two queues (each its list's next entries, in
        // order) by a bitonic merge across the wave: keys (depth bits, static
        // flag, id) are distinct and order entries as the merged index does
        // (equal depth bits: 4D first).  Queue a ascending against queue b
        // descending, lane-wise minimum (the lower half, a bitonic sequence),
        // then six half-cleaner stages sort it.
        const unsigned long long inf = ~0ull;
        const int j = 63 - lane;
        const unsigned long long ka =
            lane < na ? ((unsigned long long)s.ad[lane] << 32) | kFromStatic | s.a[lane] : inf;
        const unsigned long long kb = j < nb ? ((unsigned long long)s.bd[j] << 32) | s.b[j] : inf;
        unsigned long long m = ka < kb ? ka : kb;
#pragma unroll
        for (int st = 32; st > 0; st >>= 1) {
            const unsigned long long o = walk_xor(m, st);
            m = (lane & st) ? (m > o ? m : o) : (m < o ? m : o);
        }
        const bool act = lane < k;
        id = act ? (uint32_t)m : 0u;
        const int xa = __popcll(__ballot(act && ((uint32_t)m & kFromStatic))), xb = k - xa;
        // drop the consumed heads (every lane reads before any lane writes)
        const uint32_t ta = lane + xa < 64 ? s.a[min(lane + xa, 63)] : 0u;
        const uint32_t tad = lane + xa < 64 ? s.ad[min(lane + xa, 63)] : 0u;
        const uint32_t tb = lane + xb < 64 ? s.b[min(lane + xb, 63)] : 0u;
        const uint32_t tbd = lane + xb < 64 ? s.bd[min(lane + xb, 63)] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (lane < na - xa) {
            s.a[lane] = ta;
            s.ad[lane] = tad;
        }
        if (lane < nb - xb) {
            s.b[lane] = tb;
            s.bd[lane] = tbd;
        }
        __builtin_amdgcn_wave_barrier();
        na -= xa;
        nb -= xb;
        return k;
    }

    // Entries not yet returned (queued and still in the lists).
    __device__ uint64_t remaining() const {
        uint64_t c = walk_count(L, bit, b) + (uint64_t)nb;
        if (MERGE) c += walk_count(L, bit, a) + (uint64_t)na;
        return c;
    }

    __device__ const Rec& record(uint32_t id) const {
        return (MERGE && (id & kFromStatic)) ? recs_a[id & ~kFromStatic] : recs_b[id];
    }
};

}  // namespace h4d
